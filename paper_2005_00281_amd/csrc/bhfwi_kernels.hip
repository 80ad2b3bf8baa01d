// bhfwi_kernels.hip -- gfx950 kernels of the borehole FWI hot path.
//
// Wave-march design.  One wave64 owns a strip of 62 consecutive axial rows k
// (lanes 1..62; lanes 0 and 63 recompute the neighbours' values so that every
// z-derivative is a lane shuffle) and a chunk of radial rows i0..i1-1 that it
// marches through in increasing i, keeping the rows i-1, i, i+1 it needs in
// registers.  Each field, model and history value is read from HBM once per
// cell and step (plus one halo row per chunk and 2/64 halo lanes), every
// access is a coalesced 256-byte row segment, and no LDS or barrier is needed.
// The state is double-buffered (read buffer in, write buffer out) so that
// neighbouring waves never see half-updated rows.
//
// Forward step (Method section, Eq. 2): the velocity update and the stress
// update are fused; the velocities the stress update needs at the chunk's
// upper neighbour row are recomputed, not re-read.
// Adjoint step (Eq. 6 as the exact transpose of the discrete forward) fused
// with the zero-lag correlation of Eq. 7-8 and the illumination.
//
// Every global load is predicated on the lane's axial row being inside the
// grid (outside values are zero, the boundary convention of the scheme), and
// every store on the lane owning its cell.
#pragma once
#include "bhfwi_internal.h"

namespace bhfwi {

__device__ __forceinline__ float sh_up(float x) { return __shfl_up(x, 1, 64); }    // lane l-1
__device__ __forceinline__ float sh_dn(float x) { return __shfl_down(x, 1, 64); }  // lane l+1

__device__ __forceinline__ float ld(const float* __restrict__ p, long long idx, bool ok)
{
    return ok ? p[idx] : 0.0f;
}

// Harmonic mean of the four rigidities around a tau_rz node, zero if any is
// zero (fluid): tau_rz vanishes on the fluid-solid wall.
__device__ __forceinline__ float mu_harm(float a, float b, float c, float d)
{
    return (a > 0.f && b > 0.f && c > 0.f && d > 0.f)
               ? 4.0f * rcp(rcp(a) + rcp(b) + rcp(c) + rcp(d))
               : 0.0f;
}

// ---------------------------------------------------------------------------
// Forward step.  State block per shot (floats, relative to fst_off):
//   6 fields [vr vz trr ttt tzz trz] of NR*NZ, then 4 radial PML strips of
//   pr*NZ [A: d/dr trr at R, C: d/dr trz at Z, E: d/dr vr at C, H: d/dr vz at S],
//   then 4 axial PML strips of NR*2pz [B: d/dz trz at R, D: d/dz tzz at Z,
//   F: d/dz vz at C, G: d/dz vr at S].
//
// RU > 0: the wave's chunk has at most RU rows and every load of the chunk
// (RU + 2 rows) is issued before any arithmetic, so a wave waits for memory
// once per step instead of once per row -- the form for small grids, where
// there are too few waves to hide latency.  RU == 0: rows are loaded as the
// march reaches them (long chunks; latency hidden by occupancy).
// ---------------------------------------------------------------------------
struct FRow {
    float trr, ttt, tzz, trz, lam, mu, rho, vr, vz;
    float pA, pC, pE, pH;  // radial PML memories at this row (0 outside the layer)
    float pB, pD, pF, pG;  // axial PML memories at this row (0 outside the layer)
};

template <int RU>
__global__ void __launch_bounds__(512)
k_fwd_step(const ShotDev* __restrict__ shots, const int4* __restrict__ work, int nwork, int n,
           const float* __restrict__ lam, const float* __restrict__ mu,
           const float* __restrict__ rho, const float* __restrict__ wavelet,
           const int* __restrict__ rec_k, const float* __restrict__ pml_r,
           const float* __restrict__ pml_z, const float* __restrict__ sin,
           float* __restrict__ sout, float* __restrict__ traces, float* __restrict__ hist,
           long long cells_total)
{
    int w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    w = __builtin_amdgcn_readfirstlane(w);
    if (w >= nwork) return;
    const int lane = threadIdx.x & 63;
    const int4 wk = work[w];
    const ShotDev& S = shots[wk.x];
    if (n >= S.nt) return;

    const int NR = S.NR, NZ = S.NZ, nr = S.nr, pz = S.pz;
    const long long cells = (long long)NR * NZ;
    const int k = wk.y - 1 + lane;
    const bool kin = (k >= 0) && (k < NZ);
    const bool own = kin && lane >= 1 && lane <= kOwn;
    const bool zp = kin && (k < pz || k >= NZ - pz);
    const int kc = kin ? k : 0;
    const int kk = zp ? (k < pz ? k : k - (NZ - 2 * pz)) : 0;
    const bool top = (k + 1 >= NZ);
    const int i0 = wk.z, i1 = wk.w;
    const float dt = S.dt, idr = S.inv_dr, idz = S.inv_dz, dr = S.dr;

    const float* __restrict__ Fi = sin + S.fst_off;
    float* __restrict__ Fo = sout + S.fst_off;
    const long long oVR = 0, oVZ = cells, oTRR = 2 * cells, oTTT = 3 * cells, oTZZ = 4 * cells,
                    oTRZ = 5 * cells;
    const long long LR = S.psir_len, LZ = S.psiz_len;
    const long long oPR = 6 * cells;     // radial strips
    const long long oPZ = oPR + 4 * LR;  // axial strips
    const long long mbase = S.model_off + kc;
    const float* __restrict__ prt = pml_r + S.pml_r_off;  // [a_ri | b_ri | a_rh | b_rh] x NR
    const float* __restrict__ pzt = pml_z + S.pml_z_off;  // [a_zi | b_zi | a_zh | b_zh] x NZ
    float a_zi = 0.f, b_zi = 1.f, a_zh = 0.f, b_zh = 1.f;
    if (zp) {
        a_zi = pzt[k];
        b_zi = pzt[NZ + k];
        a_zh = pzt[2 * NZ + k];
        b_zh = pzt[3 * NZ + k];
    }
    auto ir = [&](int i) { return (long long)(i - nr) * NZ + kc; };  // radial strip index
    auto iz = [&](int i) { return (long long)i * (2 * pz) + kk; };   // axial strip index

    auto load = [&](int i) -> FRow {
        FRow X;
        X.trr = X.ttt = X.tzz = X.trz = X.lam = X.mu = X.rho = X.vr = X.vz = 0.f;
        X.pA = X.pC = X.pE = X.pH = X.pB = X.pD = X.pF = X.pG = 0.f;
        if (i < 0 || i >= NR) return X;
        const long long c = (long long)i * NZ + kc;
        X.trr = ld(Fi, oTRR + c, kin);
        X.ttt = ld(Fi, oTTT + c, kin);
        X.tzz = ld(Fi, oTZZ + c, kin);
        X.trz = ld(Fi, oTRZ + c, kin);
        X.vr = ld(Fi, oVR + c, kin);
        X.vz = ld(Fi, oVZ + c, kin);
        const long long m = mbase + (long long)i * S.model_ld;
        X.lam = ld(lam, m, kin);
        X.mu = ld(mu, m, kin);
        X.rho = ld(rho, m, kin);
        if (i >= nr) {
            const long long q = oPR + ir(i);
            X.pA = ld(Fi, q, kin);
            X.pC = ld(Fi, q + LR, kin);
            X.pE = ld(Fi, q + 2 * LR, kin);
            X.pH = ld(Fi, q + 3 * LR, kin);
        }
        if (zp) {
            const long long q = oPZ + iz(i);
            X.pB = Fi[q];
            X.pD = Fi[q + LZ];
            X.pF = Fi[q + 2 * LZ];
            X.pG = Fi[q + 3 * LZ];
        }
        return X;
    };

    float vrn0 = 0.f;               // v_r new at R(i)
    float vznm = 0.f;               // v_z new at Z(i-1)
    float mum = 0.f, mum_kp = 0.f;  // mu at row i-1, columns k and k+1

    // One march step: rows i (A) and i+1 (B) of the old state are in registers.
    auto body = [&](int i, const FRow& A, const FRow& B) {
        const int ip = i + 1;
        // ---- v_r at R(ip), ip >= 1
        float vrn1 = 0.f;
        const float trz1_km = sh_up(B.trz);
        if (ip >= 1 && ip < NR) {
            float Dr = (B.trr - A.trr) * idr;
            float Dz = (B.trz - trz1_km) * idz;
            const bool st = own && ip < i1;
            if (ip >= nr) {  // A (radial, integer position)
                const float psi = prt[NR + ip] * B.pA + prt[ip] * Dr;
                if (st) Fo[oPR + ir(ip)] = psi;
                Dr += psi;
            }
            if (zp) {  // B (axial, integer position)
                const float psi = b_zi * B.pB + a_zi * Dz;
                if (st) Fo[oPZ + iz(ip)] = psi;
                Dz += psi;
            }
            const float hoop = ((B.trr - B.ttt) + (A.trr - A.ttt)) * (0.5f * rcp(ip * dr));
            const float bR = 2.0f * rcp(A.rho + B.rho);
            vrn1 = kin ? B.vr + dt * bR * (Dr + Dz + hoop) : 0.f;
        }
        // ---- v_z at Z(i), i >= 0
        float vzn0 = 0.f;
        const float tzz0_kp = sh_dn(A.tzz);
        float rho0_kp = sh_dn(A.rho);
        if (top) rho0_kp = A.rho;
        if (i >= 0) {
            float Dr = (B.trz - A.trz) * idr;
            float Dz = (tzz0_kp - A.tzz) * idz;
            const bool st = own && i >= i0;
            if (i >= nr) {  // C (radial, half position)
                const float psi = prt[3 * NR + i] * A.pC + prt[2 * NR + i] * Dr;
                if (st) Fo[oPR + LR + ir(i)] = psi;
                Dr += psi;
            }
            if (zp) {  // D (axial, half position)
                const float psi = b_zh * A.pD + a_zh * Dz;
                if (st) Fo[oPZ + LZ + iz(i)] = psi;
                Dz += psi;
            }
            const float hoop = (B.trz + A.trz) * (0.5f * rcp((i + 0.5f) * dr));
            const float bZ = 2.0f * rcp(A.rho + rho0_kp);
            vzn0 = kin ? A.vz + dt * bZ * (Dr + Dz + hoop) : 0.f;
        }
        float mu0_kp = sh_dn(A.mu);
        if (top) mu0_kp = A.mu;
        const float vzn0_km = sh_up(vzn0);
        const float vrn0_kp = sh_dn(vrn0);
        if (i >= i0) {
            const long long c = (long long)i * NZ + kc;
            // ---- C node: normal stresses
            float err = (vrn1 - vrn0) * idr;
            const float ett = (vrn1 + vrn0) * (0.5f * rcp((i + 0.5f) * dr));
            float ezz = (vzn0 - vzn0_km) * idz;
            if (i >= nr) {  // E
                const float psi = prt[3 * NR + i] * A.pE + prt[2 * NR + i] * err;
                if (own) Fo[oPR + 2 * LR + ir(i)] = psi;
                err += psi;
            }
            if (zp) {  // F
                const float psi = b_zi * A.pF + a_zi * ezz;
                if (own) Fo[oPZ + 2 * LZ + iz(i)] = psi;
                ezz += psi;
            }
            const float tr = err + ett + ezz;
            float nrr = A.trr + dt * (A.lam * tr + 2.0f * A.mu * err);
            float ntt = A.ttt + dt * (A.lam * tr + 2.0f * A.mu * ett);
            float nzz = A.tzz + dt * (A.lam * tr + 2.0f * A.mu * ezz);
            if (i == 0 && k == S.src_k) {
                const float s = S.src_scale * wavelet[S.wave_off + n];
                nrr += s;
                ntt += s;
                nzz += s;
            }
            // ---- S node: shear stress (i >= 1)
            float nrz = 0.f;
            if (i >= 1) {
                float ez = (vrn0_kp - vrn0) * idz;
                float er = (vzn0 - vznm) * idr;
                if (zp) {  // G
                    const float psi = b_zh * A.pG + a_zh * ez;
                    if (own) Fo[oPZ + 3 * LZ + iz(i)] = psi;
                    ez += psi;
                }
                if (i >= nr) {  // H
                    const float psi = prt[NR + i] * A.pH + prt[i] * er;
                    if (own) Fo[oPR + 3 * LR + ir(i)] = psi;
                    er += psi;
                }
                nrz = A.trz + dt * mu_harm(mum, A.mu, mum_kp, mu0_kp) * (ez + er);
            }
            if (own) {
                if (i >= 1) {
                    Fo[oVR + c] = vrn0;
                    Fo[oTRZ + c] = nrz;
                }
                Fo[oVZ + c] = vzn0;
                Fo[oTRR + c] = nrr;
                Fo[oTTT + c] = ntt;
                Fo[oTZZ + c] = nzz;
                if (hist) {
                    hist[S.cell_off + c] = vrn0;
                    hist[cells_total + S.cell_off + c] = vzn0;
                }
                if (i == 0 && traces) {
                    for (int j = 0; j < S.nrec; ++j)
                        if (rec_k[S.rec_off + j] == k)
                            traces[S.trace_off + (long long)j * S.nt + n] =
                                (nrr + ntt + nzz) * (1.0f / 3.0f);
                }
            }
        }
        mum = A.mu;
        mum_kp = mu0_kp;
        vrn0 = vrn1;
        vznm = vzn0;
    };

    if constexpr (RU > 0) {
        FRow rows[RU + 2];
#pragma unroll
        for (int q = 0; q < RU + 2; ++q) rows[q] = load(i0 - 1 + q <= i1 ? i0 - 1 + q : -1);
#pragma unroll
        for (int q = 0; q < RU + 1; ++q)
            if (i0 - 1 + q < i1) body(i0 - 1 + q, rows[q], rows[q + 1]);
    } else {
        FRow A = load(i0 - 1);
        for (int i = i0 - 1; i < i1; ++i) {
            const FRow B = load(i + 1);
            body(i, A, B);
            A = B;
        }
    }
}

// ---------------------------------------------------------------------------
// Adjoint step fused with the gradient.  Adjoint state block per shot
// (relative to ast_off): 6 fields [avr avz atrr attt atzz atrz], then 5 radial
// strips [A-bar, C-bar, PhiT_r, PhiR_r, PhiH], then 5 axial strips
// [B-bar, D-bar, PhiT_z, PhiZ_z, PhiG].
//
// The adjoint of the stress-side PML memories is carried as the backward
// recursions Phi <- dt x + b Phi of the adjoint stresses x themselves, which
// give at once the transpose (through lambda Phi_T + 2 mu Phi_R) and the PML
// part of the correlation, so the gradient is exact in the PML too while only
// the velocities are stored from the forward pass.
// ---------------------------------------------------------------------------
struct ARaw {  // everything read from memory for one row
    float trr, ttt, tzz, trz, lam, mu, rho, avr, avz, vrh, vzh;
    float mu_up;  // rigidity of column k + 1 (read by the top halo lane only)
    float qA, qC, qTr, qRr, qH;  // radial strips (old)
    float qB, qD, qTz, qZz, qG;  // axial strips (old)
    float gl, gm, gs, ge;        // accumulators (rows of the chunk only)
};
struct ARow {  // derived from ARaw and the previous row's rigidity
    float trr, ttt, tzz, trz;          // adjoint stresses (residual injected)
    float rho, mu, mu_kp;              // model (mu_kp: column k+1, clamped)
    float Err, Ett, Ezz, Ez, Er;       // drivers of the transposed stress update
    float pTr, pRr, pTz, pZz, pG, pH;  // new Phi values (0 outside the PML)
};

template <int RU>
__global__ void __launch_bounds__(512)
k_adj_step(const ShotDev* __restrict__ shots, const int4* __restrict__ work, int nwork, int n,
           const float* __restrict__ lam, const float* __restrict__ mu,
           const float* __restrict__ rho, const int* __restrict__ rec_k,
           const float* __restrict__ resid, const float* __restrict__ pml_r,
           const float* __restrict__ pml_z, const float* __restrict__ ain,
           float* __restrict__ aout, const float* __restrict__ hist, float* __restrict__ acc,
           float* __restrict__ acc_rho, float* __restrict__ acc_h, float* __restrict__ wgrad,
           long long cells_total)
{
    int w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    w = __builtin_amdgcn_readfirstlane(w);
    if (w >= nwork) return;
    const int lane = threadIdx.x & 63;
    const int4 wk = work[w];
    const ShotDev& S = shots[wk.x];
    if (n >= S.nt) return;

    const int NR = S.NR, NZ = S.NZ, nr = S.nr, pz = S.pz;
    const long long cells = (long long)NR * NZ;
    const int k = wk.y - 1 + lane;
    const bool kin = (k >= 0) && (k < NZ);
    const bool own = kin && lane >= 1 && lane <= kOwn;
    const bool zp = kin && (k < pz || k >= NZ - pz);
    const int kc = kin ? k : 0;
    const int kk = zp ? (k < pz ? k : k - (NZ - 2 * pz)) : 0;
    const bool top = (k + 1 >= NZ);
    const int i0 = wk.z, i1 = wk.w;
    const float dt = S.dt, idr = S.inv_dr, idz = S.inv_dz, dr = S.dr;

    const float* __restrict__ Ai = ain + S.ast_off;
    float* __restrict__ Ao = aout + S.ast_off;
    const long long oVR = 0, oVZ = cells, oTRR = 2 * cells, oTTT = 3 * cells, oTZZ = 4 * cells,
                    oTRZ = 5 * cells;
    const long long LR = S.psir_len, LZ = S.psiz_len;
    const long long oPR = 6 * cells;
    const long long oPZ = oPR + 5 * LR;
    const long long mbase = S.model_off + kc;
    const float* __restrict__ prt = pml_r + S.pml_r_off;
    const float* __restrict__ pzt = pml_z + S.pml_z_off;
    float a_zi = 0.f, b_zi = 1.f, a_zh = 0.f, b_zh = 1.f;
    if (zp) {
        a_zi = pzt[k];
        b_zi = pzt[NZ + k];
        a_zh = pzt[2 * NZ + k];
        b_zh = pzt[3 * NZ + k];
    }
    auto ir = [&](int i) { return (long long)(i - nr) * NZ + kc; };
    auto iz = [&](int i) { return (long long)i * (2 * pz) + kk; };

    // residual of this step at receivers on this lane's row (row 0 only)
    float inj = 0.f;
    for (int j = 0; j < S.nrec; ++j)
        if (kin && rec_k[S.rec_off + j] == k)
            inj += resid[S.trace_off + (long long)j * S.nt + n] * (1.0f / 3.0f);

    const float* __restrict__ vrh = hist + S.cell_off;
    const float* __restrict__ vzh = hist + cells_total + S.cell_off;
    float* __restrict__ g_l = acc + S.cell_off;
    float* __restrict__ g_m = acc + cells_total + S.cell_off;
    float* __restrict__ g_s = acc + 2 * cells_total + S.cell_off;
    float* __restrict__ g_e = acc + 3 * cells_total + S.cell_off;

    auto load = [&](int i) -> ARaw {
        ARaw X;
        X.trr = X.ttt = X.tzz = X.trz = X.lam = X.mu = X.rho = X.avr = X.avz = X.vrh = X.vzh = 0.f;
        X.mu_up = 0.f;
        X.qA = X.qC = X.qTr = X.qRr = X.qH = X.qB = X.qD = X.qTz = X.qZz = X.qG = 0.f;
        X.gl = X.gm = X.gs = X.ge = 0.f;
        if (i < 0 || i >= NR) return X;
        const long long c = (long long)i * NZ + kc;
        X.trr = ld(Ai, oTRR + c, kin);
        X.ttt = ld(Ai, oTTT + c, kin);
        X.tzz = ld(Ai, oTZZ + c, kin);
        if (i >= 1) X.trz = ld(Ai, oTRZ + c, kin);
        X.avr = ld(Ai, oVR + c, kin);
        X.avz = ld(Ai, oVZ + c, kin);
        const long long m = mbase + (long long)i * S.model_ld;
        X.lam = ld(lam, m, kin);
        X.mu = ld(mu, m, kin);
        // the top halo lane has no lane above it to take mu[k + 1] from
        if (lane == 63) X.mu_up = ld(mu, m + 1, kin && k + 1 < NZ);
        X.rho = ld(rho, m, kin);
        X.vrh = ld(vrh, c, kin);
        X.vzh = ld(vzh, c, kin);
        if (i >= nr) {
            const long long q = oPR + ir(i);
            X.qA = ld(Ai, q, kin);
            X.qC = ld(Ai, q + LR, kin);
            X.qTr = ld(Ai, q + 2 * LR, kin);
            X.qRr = ld(Ai, q + 3 * LR, kin);
            X.qH = ld(Ai, q + 4 * LR, kin);
        }
        if (zp) {
            const long long q = oPZ + iz(i);
            X.qB = Ai[q];
            X.qD = Ai[q + LZ];
            X.qTz = Ai[q + 2 * LZ];
            X.qZz = Ai[q + 3 * LZ];
            X.qG = Ai[q + 4 * LZ];
        }
        if (i >= i0 && i < i1) {
            X.gl = ld(g_l, c, own);
            X.gm = ld(g_m, c, own);
            X.gs = ld(g_s, c, own);
            X.ge = ld(g_e, c, own);
        }
        return X;
    };

    // Drivers of the transposed stress update at row ip and the new Phi values.
    // mu_prev/_kp: rigidity of row ip-1.
    auto derive = [&](int ip, const ARaw& R, float mu_prev, float mu_prev_kp,
                      bool store) -> ARow {
        ARow X;
        X.trr = R.trr;
        X.ttt = R.ttt;
        X.tzz = R.tzz;
        X.trz = R.trz;
        X.rho = R.rho;
        X.mu = R.mu;
        X.pTr = X.pRr = X.pTz = X.pZz = X.pG = X.pH = 0.f;
        X.mu_kp = sh_dn(R.mu);
        if (lane == 63) X.mu_kp = R.mu_up;
        if (top) X.mu_kp = R.mu;
        X.Err = X.Ett = X.Ezz = X.Ez = X.Er = 0.f;
        if (ip < 0 || ip >= NR) return X;
        if (ip == 0) {
            X.trr += inj;
            X.ttt += inj;
            X.tzz += inj;
        }
        const float sa = X.trr + X.ttt + X.tzz;
        const float l = R.lam, mm2 = 2.0f * R.mu;
        X.Err = dt * (l * sa + mm2 * X.trr);
        X.Ett = dt * (l * sa + mm2 * X.ttt);
        X.Ezz = dt * (l * sa + mm2 * X.tzz);
        if (ip >= nr) {  // PhiT_r, PhiR_r at C (radial, half position)
            const float b = prt[3 * NR + ip], a = prt[2 * NR + ip];
            X.pTr = dt * sa + b * R.qTr;
            X.pRr = dt * X.trr + b * R.qRr;
            if (store) {
                Ao[oPR + 2 * LR + ir(ip)] = X.pTr;
                Ao[oPR + 3 * LR + ir(ip)] = X.pRr;
            }
            X.Err += a * (l * X.pTr + mm2 * X.pRr);
        }
        if (zp) {  // PhiT_z, PhiZ_z at C (axial, integer position)
            X.pTz = dt * sa + b_zi * R.qTz;
            X.pZz = dt * X.tzz + b_zi * R.qZz;
            if (store) {
                Ao[oPZ + 2 * LZ + iz(ip)] = X.pTz;
                Ao[oPZ + 3 * LZ + iz(ip)] = X.pZz;
            }
            X.Ezz += a_zi * (l * X.pTz + mm2 * X.pZz);
        }
        if (ip >= 1) {
            const float muS = mu_harm(mu_prev, R.mu, mu_prev_kp, X.mu_kp);
            const float s = dt * muS * X.trz;
            X.Ez = s;
            X.Er = s;
            if (zp) {  // PhiG at S (axial, half position)
                X.pG = dt * X.trz + b_zh * R.qG;
                if (store) Ao[oPZ + 4 * LZ + iz(ip)] = X.pG;
                X.Ez += a_zh * muS * X.pG;
            }
            if (ip >= nr) {  // PhiH at S (radial, integer position)
                X.pH = dt * X.trz + prt[NR + ip] * R.qH;
                if (store) Ao[oPR + 4 * LR + ir(ip)] = X.pH;
                X.Er += prt[ip] * muS * X.pH;
            }
        }
        if (!kin) X.Err = X.Ett = X.Ezz = X.Ez = X.Er = 0.f;
        return X;
    };

    // carried between rows: R(i) [aDr, aDzR, hR], Z(i-1) contribution zm,
    // v_z history of row i-1
    float R0_aDr = 0.f, R0_aDzR = 0.f, R0_hR = 0.f, zm = 0.f, vzhm = 0.f;

    // One march step: raw rows i (P) and i+1 (Q), derived rows X0 (i), X1 (i+1).
    auto body = [&](int i, const ARaw& P, const ARaw& Q, const ARow& X0, const ARow& X1) {
        const int ip = i + 1;
        const bool own_ip = own && ip >= i0 && ip < i1;
        const bool own_i = own && i >= i0;
        // ---- R(ip): transposed stress update into avr, then transposed velocity update
        float R1_aDr = 0.f, R1_aDzR = 0.f, R1_hR = 0.f;
        const float Ez1_km = sh_up(X1.Ez);
        if (ip >= 1 && ip < NR) {
            const long long c = (long long)ip * NZ + kc;
            // the increment first: the density correlation needs it unrounded
            const float dar = (X0.Err - X1.Err) * idr + X0.Ett * (0.5f * rcp((ip - 0.5f) * dr)) +
                              X1.Ett * (0.5f * rcp((ip + 0.5f) * dr)) + (Ez1_km - X1.Ez) * idz;
            const float avr = Q.avr + dar;
            const float W = kin ? dt * (2.0f * rcp(X0.rho + X1.rho)) * avr : 0.f;
            float aDr = W, aDz = W;
            if (ip >= nr) {  // A-bar
                const float qv = Q.qA + W;
                if (own_ip) Ao[oPR + ir(ip)] = prt[NR + ip] * qv;
                aDr += prt[ip] * qv;
            }
            if (zp) {  // B-bar
                const float qv = Q.qB + W;
                if (own_ip) Ao[oPZ + iz(ip)] = b_zi * qv;
                aDz += a_zi * qv;
            }
            if (own_ip) Ao[oVR + c] = avr;
            // density correlation (optional): increment of a_v times v^{n+1/2}
            if (acc_rho && own_ip) acc_rho[S.cell_off + c] += dar * Q.vrh;
            R1_aDr = aDr;
            R1_aDzR = aDz;
            R1_hR = W * (0.5f * rcp(ip * dr));
        }
        // ---- Z(i)
        float Z_aDrZ = 0.f, Z_WZ = 0.f, Z_aDzZ = 0.f;
        const float Ezz0_kp = sh_dn(X0.Ezz);
        float rho0_kp = sh_dn(X0.rho);
        if (top) rho0_kp = X0.rho;
        if (i >= 0) {
            const long long c = (long long)i * NZ + kc;
            const float daz = (X0.Ezz - Ezz0_kp) * idz + (X0.Er - X1.Er) * idr;
            const float avz = P.avz + daz;
            const float W = kin ? dt * (2.0f * rcp(X0.rho + rho0_kp)) * avz : 0.f;
            float aDr = W, aDz = W;
            if (i >= nr) {  // C-bar (radial, half position)
                const float qv = P.qC + W;
                if (own_i) Ao[oPR + LR + ir(i)] = prt[3 * NR + i] * qv;
                aDr += prt[2 * NR + i] * qv;
            }
            if (zp) {  // D-bar (axial, half position)
                const float qv = P.qD + W;
                if (own_i) Ao[oPZ + LZ + iz(i)] = b_zh * qv;
                aDz += a_zh * qv;
            }
            if (own_i) Ao[oVZ + c] = avz;
            if (acc_rho && own_i) acc_rho[cells_total + S.cell_off + c] += daz * P.vzh;
            Z_aDrZ = aDr;
            Z_WZ = W;
            Z_aDzZ = aDz;
        }
        const float aDzZ_km = sh_up(Z_aDzZ);
        const float aDzR_kp = sh_dn(R0_aDzR);
        const float vrh0 = P.vrh, vrh1 = Q.vrh, vzh0 = P.vzh;
        const float vzh0_km = sh_up(vzh0);
        const float vrh0_kp = sh_dn(vrh0);
        if (i >= i0) {
            const long long c = (long long)i * NZ + kc;
            const float nrr = X0.trr + R0_aDr * idr + R0_hR - R1_aDr * idr + R1_hR;
            const float ntt = X0.ttt - R0_hR - R1_hR;
            const float nzz = X0.tzz - Z_aDzZ * idz + aDzZ_km * idz;
            const float rh = (i + 0.5f) * dr;
            float nrz = 0.f;
            if (i >= 1)
                nrz = X0.trz + (R0_aDzR - aDzR_kp) * idz - Z_aDrZ * idr + Z_WZ * (0.5f * rcp(rh)) + zm;
            // Eq. 7-8: correlate the strain rates of v^{n+1/2} with dJ/dtau^{n+1}
            const float err = (vrh1 - vrh0) * idr;
            const float ett = (vrh1 + vrh0) * (0.5f * rcp(rh));
            const float ezz = (vzh0 - vzh0_km) * idz;
            const float sa = X0.trr + X0.ttt + X0.tzz;
            // source wavelet gradient (optional): dJ/dw[n] = src_scale dJ/dtau^{n+1}
            if (wgrad && own && i == 0 && k == S.src_k) wgrad[S.wave_off + n] = S.src_scale * sa;
            float dgl = dt * (err + ett + ezz) * sa;
            float dgm = 2.0f * dt * (err * X0.trr + ett * X0.ttt + ezz * X0.tzz);
            if (i >= nr) {
                const float a = prt[2 * NR + i];
                dgl += a * err * X0.pTr;
                dgm += 2.0f * a * err * X0.pRr;
            }
            if (zp) {
                dgl += a_zi * ezz * X0.pTz;
                dgm += 2.0f * a_zi * ezz * X0.pZz;
            }
            const float ur = 0.5f * (vrh0 + vrh1), uz = 0.5f * (vzh0_km + vzh0);
            const float dge = dt * (ur * ur + uz * uz);
            float dgs = 0.f, es = 0.f;
            if (i >= 1) {
                const float ez = (vrh0_kp - vrh0) * idz;
                const float er = (vzh0 - vzhm) * idr;
                es = ez + er;
                dgs = dt * (ez + er) * X0.trz;
                if (zp) dgs += a_zh * ez * X0.pG;
                if (i >= nr) dgs += prt[i] * er * X0.pH;
            }
            // virtual-source pseudo-Hessian diagonal (optional)
            if (acc_h && own) {
                const float dv = err + ett + ezz;
                acc_h[S.cell_off + c] += dt * dt * (3.0f * dv * dv);
                acc_h[cells_total + S.cell_off + c] +=
                    dt * dt * (4.0f * (err * err + ett * ett + ezz * ezz) + es * es);
            }
            if (own) {
                Ao[oTRR + c] = nrr;
                Ao[oTTT + c] = ntt;
                Ao[oTZZ + c] = nzz;
                if (i >= 1) {
                    Ao[oTRZ + c] = nrz;
                    g_s[c] = P.gs + dgs;
                }
                g_l[c] = P.gl + dgl;
                g_m[c] = P.gm + dgm;
                g_e[c] = P.ge + dge;
            }
        }
        zm = (i >= 0) ? Z_aDrZ * idr + Z_WZ * (0.5f * rcp((i + 0.5f) * dr)) : 0.f;
        R0_aDr = R1_aDr;
        R0_aDzR = R1_aDzR;
        R0_hR = R1_hR;
        vzhm = vzh0;
    };

    // rigidity of row i0-2, needed for the shear drivers of row i0-1
    float mpp = 0.f, mpp_kp = 0.f;
    if (i0 >= 2) mpp = ld(mu, mbase + (long long)(i0 - 2) * S.model_ld, kin);
    mpp_kp = sh_dn(mpp);
    if (lane == 63)
        mpp_kp = i0 >= 2 ? ld(mu, mbase + (long long)(i0 - 2) * S.model_ld + 1, kin && k + 1 < NZ)
                         : 0.f;
    if (top) mpp_kp = mpp;

    if constexpr (RU > 0) {
        ARaw raw[RU + 2];
#pragma unroll
        for (int q = 0; q < RU + 2; ++q) raw[q] = load(i0 - 1 + q <= i1 ? i0 - 1 + q : -1);
        ARow X0 = derive(i0 - 1, raw[0], mpp, mpp_kp, false);
#pragma unroll
        for (int q = 0; q < RU + 1; ++q) {
            const int i = i0 - 1 + q;
            if (i < i1) {
                const ARow X1 = derive(i + 1, raw[q + 1], X0.mu, X0.mu_kp,
                                       own && i + 1 >= i0 && i + 1 < i1);
                body(i, raw[q], raw[q + 1], X0, X1);
                X0 = X1;
            }
        }
    } else {
        ARaw P = load(i0 - 1);
        ARow X0 = derive(i0 - 1, P, mpp, mpp_kp, false);
        for (int i = i0 - 1; i < i1; ++i) {
            const ARaw Q = load(i + 1);
            const ARow X1 = derive(i + 1, Q, X0.mu, X0.mu_kp, own && i + 1 >= i0 && i + 1 < i1);
            body(i, P, Q, X0, X1);
            P = Q;
            X0 = X1;
        }
    }
}

// ---------------------------------------------------------------------------
// Small kernels
// ---------------------------------------------------------------------------
__global__ void k_fill(float* __restrict__ p, long long n, float v)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = v;
}

__global__ void k_moduli(long long n, const float* __restrict__ vp, const float* __restrict__ vs,
                         const float* __restrict__ rho, float* __restrict__ lam,
                         float* __restrict__ mu)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float r = rho[i], p = vp[i], s = vs[i];
        const float m = r * s * s;
        lam[i] = r * p * p - 2.0f * m;
        mu[i] = m;
    }
}

__global__ void k_moduli_grad(long long n, const float* __restrict__ vp,
                              const float* __restrict__ vs, const float* __restrict__ rho,
                              const float* __restrict__ g_lam, const float* __restrict__ g_mu,
                              float* __restrict__ g_vp, float* __restrict__ g_vs,
                              float* __restrict__ g_rho)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float r2 = 2.0f * rho[i], gl = g_lam[i], gm = g_mu[i];
        const float a = vp[i], b = vs[i];
        g_vp[i] = r2 * a * gl;
        g_vs[i] = r2 * b * (gm - 2.0f * gl);
        if (g_rho) g_rho[i] = (a * a - 2.0f * b * b) * gl + b * b * gm;
    }
}

__global__ void k_velocities(long long n, const float* __restrict__ lam,
                             const float* __restrict__ mu, const float* __restrict__ rho,
                             float* __restrict__ vp, float* __restrict__ vs)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float r = rho[i];
        vp[i] = sqrtf((lam[i] + 2.0f * mu[i]) / r);
        vs[i] = sqrtf(mu[i] / r);
    }
}

// Deterministic two-level sum of 0.5 (d - obs)^2 in double; resid = d - obs.
__global__ void __launch_bounds__(256)
k_misfit_partial(long long n, const float* __restrict__ d, const float* __restrict__ obs,
                 float* __restrict__ resid, double* __restrict__ part)
{
    __shared__ double sh[256];
    double s = 0.0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float r = d[i] - obs[i];
        resid[i] = r;
        s += 0.5 * (double)r * (double)r;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Sum of np partials into *out (or added to it).  With status != nullptr a
// non-finite sum raises status[0] to 1.
__global__ void __launch_bounds__(256)
k_sum_partials(int np, const double* __restrict__ part, double* __restrict__ out, int add,
               int* __restrict__ status)
{
    __shared__ double sh[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) s += part[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *out = add ? *out + sh[0] : sh[0];
        if (status && !isfinite(sh[0])) status[0] = 1;
    }
}

// Add one shot's accumulators into the global grids; folds the tau_rz-node
// rigidity gradient into the C cells: d muS / d mu_c = muS^2 / (4 mu_c^2) for
// every occurrence of c among the four cells around the node.
__global__ void k_finalize_shot(const ShotDev* __restrict__ shots, int s,
                                const float* __restrict__ mu, const float* __restrict__ acc,
                                long long cells_total, float* __restrict__ g_lam,
                                float* __restrict__ g_mu, float* __restrict__ illum)
{
    const ShotDev& S = shots[s];
    const int NR = S.NR, NZ = S.NZ;
    const long long cells = (long long)NR * NZ;
    const float* gl = acc + S.cell_off;
    const float* gm = acc + cells_total + S.cell_off;
    const float* gs = acc + 2 * cells_total + S.cell_off;
    const float* ge = acc + 3 * cells_total + S.cell_off;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += stride) {
        const int i = (int)(c / NZ), k = (int)(c % NZ);
        const long long m = S.model_off + (long long)i * S.model_ld + k;
        auto M = [&](int ii, int kk2) {
            return mu[S.model_off + (long long)ii * S.model_ld + kk2];
        };
        const float mc = mu[m];
        float fold = 0.f;
        if (mc > 0.f) {
            for (int ii = i; ii <= i + 1; ++ii) {
                if (ii < 1 || ii >= NR) continue;
                for (int kp = k - 1; kp <= k; ++kp) {
                    if (kp < 0) continue;
                    const int k1 = (kp + 1 < NZ) ? kp + 1 : NZ - 1;
                    const float muS = mu_harm(M(ii - 1, kp), M(ii, kp), M(ii - 1, k1), M(ii, k1));
                    if (!(muS > 0.f)) continue;
                    const float wgt = (kp == k) ? ((k1 == k) ? 2.0f : 1.0f) : 1.0f;
                    fold += wgt * gs[(long long)ii * NZ + kp] * muS * muS / (4.0f * mc * mc);
                }
            }
        }
        g_lam[m] += gl[c];
        g_mu[m] += gm[c] + fold;
        illum[m] += ge[c];
    }
}

// Add one shot's density correlation into the global dJ/drho.  acc_rho holds
// b dJ/db at the R nodes (plane 0) and the Z nodes (plane 1); with
// b_R = 2/(rho[i-1,k] + rho[i,k]) and b_Z = 2/(rho[i,k] + rho[i,k1])
// (k1 = min(k+1, NZ-1)) each node adds -(b/2) (b dJ/db) to both of its cells.
// Gathered per cell, so no atomics: the R nodes (i,k) and (i+1,k), the Z
// nodes (i,k) and (i,k-1); on the top row k1 = k and the own Z node counts
// twice.
__global__ void k_finalize_rho_shot(const ShotDev* __restrict__ shots, int s,
                                    const float* __restrict__ rho,
                                    const float* __restrict__ acc_rho, long long cells_total,
                                    float* __restrict__ g_rho)
{
    const ShotDev& S = shots[s];
    const int NR = S.NR, NZ = S.NZ;
    const long long cells = (long long)NR * NZ;
    const float* sR = acc_rho + S.cell_off;
    const float* sZ = acc_rho + cells_total + S.cell_off;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += stride) {
        const int i = (int)(c / NZ), k = (int)(c % NZ);
        auto R = [&](int ii, int kk) {
            return rho[S.model_off + (long long)ii * S.model_ld + kk];
        };
        const float r0 = R(i, k);
        float g = 0.f;
        if (i >= 1) g -= sR[c] / (R(i - 1, k) + r0);
        if (i + 1 < NR) g -= sR[c + NZ] / (r0 + R(i + 1, k));
        const int k1 = (k + 1 < NZ) ? k + 1 : k;
        g -= (k1 == k ? 2.0f : 1.0f) * sZ[c] / (r0 + R(i, k1));
        if (k >= 1) g -= sZ[c - 1] / (R(i, k - 1) + r0);
        g_rho[S.model_off + (long long)i * S.model_ld + k] += g;
    }
}

// Add two per-shot planes (src, src + cells_total) of one shot's window into
// the global grids d0, d1.
__global__ void k_window_add2(const ShotDev* __restrict__ shots, int s,
                              const float* __restrict__ src, long long cells_total,
                              float* __restrict__ d0, float* __restrict__ d1)
{
    const ShotDev& S = shots[s];
    const int NZ = S.NZ;
    const long long cells = (long long)S.NR * NZ;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += stride) {
        const long long m = S.model_off + (c / NZ) * S.model_ld + (c % NZ);
        d0[m] += src[S.cell_off + c];
        d1[m] += src[cells_total + S.cell_off + c];
    }
}

// Block-wise maxima over mask cells of up to four arrays (|x|), written as
// non-negative floats to part[4 * block + q].
__global__ void __launch_bounds__(256)
k_absmax_partial(long long n, const uint8_t* __restrict__ mask, const float* __restrict__ a0,
                 const float* __restrict__ a1, const float* __restrict__ a2,
                 const float* __restrict__ a3, float* __restrict__ part)
{
    __shared__ float sh[4][256];
    float m[4] = {0.f, 0.f, 0.f, 0.f};
    const float* a[4] = {a0, a1, a2, a3};
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (!mask[i]) continue;
        for (int q = 0; q < 4; ++q)
            if (a[q]) m[q] = fmaxf(m[q], fabsf(a[q][i]));
    }
    for (int q = 0; q < 4; ++q) sh[q][threadIdx.x] = m[q];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int q = 0; q < 4; ++q)
                sh[q][threadIdx.x] = fmaxf(sh[q][threadIdx.x], sh[q][threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x < 4) part[4 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

__device__ float reduce_part_max(const float* __restrict__ part, int np, int q, float* sh)
{
    float m = 0.f;
    for (int b = threadIdx.x; b < np; b += blockDim.x) m = fmaxf(m, part[4 * b + q]);
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    const float r = sh[0];
    __syncthreads();
    return r;
}

// Scales both gradients by P = 1/(E + eps max E) on mask cells (0 elsewhere).
// With dot != nullptr also writes the block sums of g . P g (both
// parameters, double) to dot[blockIdx.x]: the directional derivative of the
// misfit along the preconditioned step, used by the line search.
__global__ void __launch_bounds__(256)
k_precond_apply(long long n, const uint8_t* __restrict__ mask, const float* __restrict__ illum,
                float eps, const float* __restrict__ part, int np, float* __restrict__ g_lam,
                float* __restrict__ g_mu, double* __restrict__ dot)
{
    __shared__ float sh[256];
    __shared__ double shd[256];
    const float emax = reduce_part_max(part, np, 0, sh);
    double s = 0.0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (!mask[i]) {
            g_lam[i] = 0.f;
            g_mu[i] = 0.f;
            continue;
        }
        const float p = 1.0f / (illum[i] + eps * emax);
        const float gl = g_lam[i], gm = g_mu[i];
        g_lam[i] = gl * p;
        g_mu[i] = gm * p;
        s += (double)p * ((double)gl * gl + (double)gm * gm);
    }
    if (!dot) return;  // uniform
    shd[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) shd[threadIdx.x] += shd[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) dot[blockIdx.x] = shd[0];
}

// One gradient scaled by P = w[row] / (d + eps max d) on mask cells (0
// elsewhere); d (nullable: P without it is w alone) is a diagonal such as the
// illumination or a pseudo-Hessian, w (nullable) a weight per radial row of
// ld elements.  dot (nullable) receives the block sums of g . P g.
__global__ void __launch_bounds__(256)
k_precond_diag_apply(long long n, int ld, const uint8_t* __restrict__ mask,
                     const float* __restrict__ diag, const float* __restrict__ roww, float eps,
                     const float* __restrict__ part, int np, float* __restrict__ g,
                     double* __restrict__ dot)
{
    __shared__ float sh[256];
    __shared__ double shd[256];
    const float dmax = diag ? reduce_part_max(part, np, 0, sh) : 0.f;
    double s = 0.0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (!mask[i]) {
            g[i] = 0.f;
            continue;
        }
        float p = diag ? 1.0f / (diag[i] + eps * dmax) : 1.0f;
        if (roww) p *= roww[i / ld];
        const float gi = g[i];
        g[i] = gi * p;
        s += (double)p * ((double)gi * gi);
    }
    if (!dot) return;  // uniform
    shd[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) shd[threadIdx.x] += shd[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) dot[blockIdx.x] = shd[0];
}

// Radial taper per row of C cells, r = (i + 1/2) dr: 0 inside r0, a sin^2
// ramp to 1 at r1, 1 beyond.
__global__ void k_radial_taper(int nrow, float dr, float r0, float r1, float* __restrict__ w)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrow) return;
    const float r = (i + 0.5f) * dr;
    const float x = fminf(fmaxf((r - r0) / fmaxf(r1 - r0, 1e-30f), 0.f), 1.f);
    const float s = sinf(0.5f * 3.14159265358979f * x);
    w[i] = s * s;
}

// Density step with its own greatest-change rule: alpha = eta max|rho| /
// max|g| over mask cells (part: block maxima of |g| in slot 0 and of rho in
// slot 1), rho <- clamp(rho - alpha g, rho_min, rho_max) on mask cells.
__global__ void __launch_bounds__(256)
k_update_density_apply(long long n, const uint8_t* __restrict__ mask, float* __restrict__ rho,
                       const float* __restrict__ g, const float* __restrict__ part, int np,
                       float eta, float rho_min, float rho_max, float* __restrict__ alpha_out)
{
    __shared__ float sh[256];
    const float gmax = reduce_part_max(part, np, 0, sh);
    const float rmax = reduce_part_max(part, np, 1, sh);
    const float alpha = gmax > 0.f ? eta * rmax / gmax : 0.f;
    if (alpha_out && blockIdx.x == 0 && threadIdx.x == 0) *alpha_out = alpha;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (!mask[i]) continue;
        rho[i] = fminf(fmaxf(rho[i] - alpha * g[i], rho_min), rho_max);
    }
}

// Step length of the parabolic line search.  With the misfit J0 at the
// current model, J1 at the trial step alpha1 and the slope -gpg of J along
// the preconditioned step at alpha = 0, the parabola
//   J(a) = J0 - gpg a + c a^2,   c = (J1 - J0 + gpg alpha1) / alpha1^2
// has its minimum at gpg / (2c) when c > 0; that value is kept inside
// [alpha1/10, 3 alpha1].  Without a minimum (c <= 0) the trial step is kept
// if it lowered the misfit and halved otherwise.  One thread.
__global__ void k_line_search(const double* __restrict__ J0, const double* __restrict__ J1,
                              const double* __restrict__ gpg, const float* __restrict__ alpha1,
                              float* __restrict__ alpha_out)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const double a1 = alpha1[0], j0 = J0[0], j1 = J1[0], g = gpg[0];
    double a = 0.0;
    if (a1 > 0.0) {
        const double c = (j1 - j0 + g * a1) / (a1 * a1);
        if (c > 0.0)
            a = fmin(fmax(g / (2.0 * c), 0.1 * a1), 3.0 * a1);
        else
            a = (j1 <= j0) ? a1 : 0.5 * a1;
    }
    alpha_out[0] = (float)a;
}

// part holds the maxima of |g_lam|, |g_mu|, |lam|, |mu| over mask cells.
__global__ void __launch_bounds__(256)
k_update_apply(long long n, const uint8_t* __restrict__ mask, float* __restrict__ lam,
               float* __restrict__ mu, const float* __restrict__ rho,
               const float* __restrict__ g_lam, const float* __restrict__ g_mu,
               const float* __restrict__ part, int np, float eta, float alpha_override,
               const float* __restrict__ alpha_in, float vp_min, float vp_max, float vs_min,
               float vs_max, float* __restrict__ alpha_out)
{
    __shared__ float sh[256];
    float alpha = alpha_in ? alpha_in[0] : alpha_override;
    if (!alpha_in && !(alpha > 0.f)) {
        const float gl = reduce_part_max(part, np, 0, sh);
        const float gm = reduce_part_max(part, np, 1, sh);
        const float lm = reduce_part_max(part, np, 2, sh);
        const float mm = reduce_part_max(part, np, 3, sh);
        const float rl = lm > 0.f ? gl / lm : 0.f, rm = mm > 0.f ? gm / mm : 0.f;
        const float r = fmaxf(rl, rm);
        alpha = r > 0.f ? eta / r : 0.f;
    }
    if (alpha_out && blockIdx.x == 0 && threadIdx.x == 0) *alpha_out = alpha;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (!mask[i]) continue;
        const float r = rho[i];
        float m = mu[i] - alpha * g_mu[i];
        float l = lam[i] - alpha * g_lam[i];
        m = fminf(fmaxf(m, r * vs_min * vs_min), r * vs_max * vs_max);
        float p = l + 2.0f * m;
        p = fminf(fmaxf(p, r * vp_min * vp_min), r * vp_max * vp_max);
        lam[i] = p - 2.0f * m;
        mu[i] = m;
    }
}

}  // namespace bhfwi
