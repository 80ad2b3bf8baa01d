// bhfwi_tb_fwd.hip -- temporally blocked forward step (Method section, Eq. 2).
//
// One workgroup of W wave64 owns a tile of TR = TRE - 2T radial
// rows by TZ = 64 - 2T axial rows and advances it T time steps per launch
// (of those rows it writes back the ones from the tile table's fourth entry
// up: a tile whose window overlaps the one below it leaves their rows to it).
// It loads the tile plus a T-cell halo on every side (TRE rows x 64 columns,
// lane = column), keeps each cell's six fields, its precomputed medium
// coefficients and its PML memories in registers (thread (wave w, lane l)
// holds rows w, w+W, ..., so a row index is uniform over a wave), and shares
// the fields through LDS (with a zeroed guard row above and below) for the
// radial neighbour reads; axial neighbours are lanes of the same wave, read
// with DPP wavefront shifts.  Every step needs the neighbours' previous values, so the
// correct region shrinks by one cell per step on every side; after T steps it
// is exactly the owned tile, which is all that is written back.  State
// crosses HBM once per T steps instead of once per step.  Rows that have
// fallen out of the correct region are skipped (whole-wave branches), which
// trims the halo recomputation by about T (T - 1) of T TRE row-steps.
//
// The step loop has no per-cell branches: cells outside the grid, v_r and
// tau_rz on the axis and the non-source cells carry zero coefficients, so the
// same arithmetic leaves them at zero.  The PML memories are updated only in
// the instantiations of the loop used by tiles that touch a PML layer, and
// only those of the layers (radial, axial) the tile reaches.
#pragma once
#include "bhfwi_internal.h"

namespace bhfwi {

template <int V>
struct IntC {
    static constexpr int value = V;
};

template <int T, int TRE, int W, int PM>
__global__ void __launch_bounds__(64 * W, (W >= 16 && (TRE == W || (PM == 0 && TRE <= 3 * W))) ? 8 : 1)
k_fwd_tb(const ShotDev* __restrict__ shots, const int4* __restrict__ work, int nwork, int map,
         int n0,
         int nsteps, const float* __restrict__ lam, const float* __restrict__ mu,
         const float* __restrict__ rho, const float* __restrict__ wavelet,
         const int* __restrict__ rec_k, const float* __restrict__ pml_r,
         const float* __restrict__ pml_z, const float* __restrict__ sin,
         float* __restrict__ sout, float* __restrict__ traces, float* __restrict__ hist,
         long long hist_stride, long long cells_total)
{
    static_assert(TRE % W == 0 && TRE > 2 * T && 64 > 2 * T, "tile too small for the halo");
    constexpr int RPT = TRE / W;  // rows per thread
    constexpr int LDW = (TRE + 2) * 64;   // one LDS plane with guard rows
    enum { TRR = 0, TTT, TRZ, VR, VZ, NPL };
    __shared__ float L[NPL][LDW];
    __shared__ float Lwav[T];  // source samples of this launch's steps

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

    const float* __restrict__ Fi = sin + S.fst_off;
    float* __restrict__ Fo = sout + S.fst_off;
    const long long LR = S.psir_len, LZ = S.psiz_len;
    const long long oPR = 6 * cells, oPZ = oPR + 4 * LR;
    const float* __restrict__ prt = pml_r + S.pml_r_off;
    const float* __restrict__ pzt = pml_z + S.pml_z_off;

    if (wave == 0) {
#pragma unroll
        for (int f = 0; f < NPL; ++f) {
            L[f][lane] = 0.f;
            L[f][(TRE + 1) * 64 + lane] = 0.f;
        }
        if (lane < T) Lwav[lane] = lane < ns ? wavelet[S.wave_off + n0 + lane] : 0.f;
    }
    // receiver recorded by this lane's axial row (first match), or -1
    int rj = -1;
    if (traces && wk.z == 0)
        for (int r = S.nrec - 1; r >= 0; --r)
            if (kin && rec_k[S.rec_off + r] == k) rj = r;

    // per cell (registers) and per row (wave-uniform) state
    float vr[RPT], vz[RPT], trr[RPT], ttt[RPT], tzz[RPT], trz[RPT];
    float cl[RPT], c2m[RPT], dbR[RPT], dbZ[RPT], dmuS[RPT], srcw[RPT];
    float rR[RPT], rZ[RPT];  // 1/(2 r) at R and C/Z nodes (0 on the axis / outside)
    float pA[RPT], pB[RPT], pC[RPT], pD[RPT], pE[RPT], pF[RPT], pG[RPT], pH[RPT];
    float a_ri[RPT], b_ri[RPT], a_rh[RPT], b_rh[RPT];
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
        const long long c = (long long)(iin ? i : 0) * NZ + kc;
        vr[j] = in ? Fi[c] : 0.f;
        vz[j] = in ? Fi[cells + c] : 0.f;
        trr[j] = in ? Fi[2 * cells + c] : 0.f;
        ttt[j] = in ? Fi[3 * cells + c] : 0.f;
        tzz[j] = in ? Fi[4 * cells + c] : 0.f;
        trz[j] = in ? Fi[5 * cells + c] : 0.f;
        const long long m = S.model_off + (long long)(iin ? i : 0) * S.model_ld;
        const long long mm = m - S.model_ld;  // row i-1
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
        srcw[j] = (in && i == 0 && k == S.src_k) ? S.src_scale : 0.f;
        rR[j] = wave_uniform((iin && i >= 1) ? 0.5f * rcp(i * dr) : 0.f);
        rZ[j] = wave_uniform(iin ? 0.5f * rcp((i + 0.5f) * dr) : 0.f);
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
        const int x = (e + 1) * 64 + lane;
        L[TRR][x] = trr[j];
        L[TTT][x] = ttt[j];
        L[TRZ][x] = trz[j];
        L[VR][x] = vr[j];
        L[VZ][x] = vz[j];
    }
    __syncthreads();

    // byte offset of this lane's cell in each row within a history plane
    unsigned hoff[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int i = wk.z - T + wave + W * j;
        hoff[j] = (unsigned)(max(i, 0) * NZ + kc) * 4u;
    }
    // Rows that still matter at step t: the correct region shrinks one row
    // per step on each side, so after step t only rows t + 1 .. TRE - t - 2
    // hold correct values, and they read rows t .. TRE - t - 1 of this step.
    // Rows e < t and e >= TRE - t are skipped (the test is uniform over a
    // wave); a row that reads one of them is itself discarded after the step.
    auto live = [&](int e, int t) { return e >= t && e < TRE - t; };

    // The step loop in three PML forms besides the plain one: radial and
    // axial memories, radial only, axial only.  A tile that does not reach a
    // layer has zero coefficients for it everywhere, so leaving that layer's
    // terms out changes nothing; most PML tiles reach the radial layer only.
    auto steps = [&](auto PRC, auto PZC) {
        constexpr bool PR = decltype(PRC)::value != 0, PZ = decltype(PZC)::value != 0;
        for (int t = 0; t < ns; ++t) {
            const int n = n0 + t;
            const float wv = Lwav[t];
            // this step's history planes (uniform base; per-row byte offsets)
            char* const hvr_t =
                hist ? reinterpret_cast<char*>(hist + (long long)t * hist_stride + S.cell_off)
                     : nullptr;
            char* const hvz_t = hist ? hvr_t + 4 * cells_total : nullptr;
            // ---- velocities (R and Z nodes) from the stresses
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                if (!live(wave + W * j, t)) continue;  // uniform
                const int x = (wave + W * j + 1) * 64 + lane;
                const float trr_m = L[TRR][x - 64], ttt_m = L[TTT][x - 64];
                const float trz_km = from_lane_below(trz[j]), trz_ip = L[TRZ][x + 64];
                const float tzz_kp = from_lane_above(tzz[j]);
                float Dr = (trr[j] - trr_m) * idr;
                float Dz = (trz[j] - trz_km) * idz;
                float Dr2 = (trz_ip - trz[j]) * idr;
                float Dz2 = (tzz_kp - tzz[j]) * idz;
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
                vr[j] += dbR[j] * (Dr + Dz + ((trr[j] - ttt[j]) + (trr_m - ttt_m)) * rR[j]);
                vz[j] += dbZ[j] * (Dr2 + Dz2 + (trz_ip + trz[j]) * rZ[j]);
                L[VR][x] = vr[j];
                L[VZ][x] = vz[j];
            }
            __syncthreads();
            // ---- stresses (C and S nodes) from the new velocities
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                const int e = wave + W * j;
                if (!live(e, t)) continue;  // uniform
                const int x = (e + 1) * 64 + lane;
                const float vr_ip = L[VR][x + 64], vz_km = from_lane_below(vz[j]);
                const float vr_kp = from_lane_above(vr[j]), vz_im = L[VZ][x - 64];
                float err = (vr_ip - vr[j]) * idr;
                const float ett = (vr_ip + vr[j]) * rZ[j];
                float ezz = (vz[j] - vz_km) * idz;
                float ez = (vr_kp - vr[j]) * idz;
                float er = (vz[j] - vz_im) * idr;
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
                L[TRR][x] = trr[j];
                L[TTT][x] = ttt[j];
                L[TRZ][x] = trz[j];
                const int i = wk.z - T + e;
                const bool own = kin && lown && e >= T && e < TRE - T && i >= wk.w && i < NR;
                if (hist && own) {
                    // streamed out, read back segments later: not kept in L2
                    __builtin_nontemporal_store(vr[j], reinterpret_cast<float*>(hvr_t + hoff[j]));
                    __builtin_nontemporal_store(vz[j], reinterpret_cast<float*>(hvz_t + hoff[j]));
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
        const int i = wk.z - T + e;
        const bool in = kin && i >= 0 && i < NR;
        if (!(in && lown && e >= T && e < TRE - T && i >= wk.w)) continue;
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

}  // namespace bhfwi
