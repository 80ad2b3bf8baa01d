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
               ? 4.0f / (1.0f / a + 1.0f / b + 1.0f / c + 1.0f / d)
               : 0.0f;
}

// ---------------------------------------------------------------------------
// Forward step.  State block per shot (floats, relative to fst_off):
//   6 fields [vr vz trr ttt tzz trz] of NR*NZ, then 4 radial PML strips of
//   pr*NZ [A: d/dr trr at R, C: d/dr trz at Z, E: d/dr vr at C, H: d/dr vz at S],
//   then 4 axial PML strips of NR*2pz [B: d/dz trz at R, D: d/dz tzz at Z,
//   F: d/dz vz at C, G: d/dz vr at S].
// ---------------------------------------------------------------------------
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
    const long long oPR = 6 * cells;                       // radial strips
    const long long oPZ = oPR + 4LL * S.psir_len;          // axial strips
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
    auto ir = [&](int i) { return (long long)(i - nr) * NZ + kc; };      // radial strip index
    auto iz = [&](int i) { return (long long)i * (2 * pz) + kk; };       // axial strip index

    // registers of row i (old state and model) and of the velocities already updated
    float trr0 = 0.f, ttt0 = 0.f, tzz0 = 0.f, trz0 = 0.f, lam0 = 0.f, mu0 = 0.f, rho0 = 0.f;
    float vrn0 = 0.f;            // v_r new at R(i)
    float vznm = 0.f;            // v_z new at Z(i-1)
    float mum = 0.f, mum_kp = 0.f;  // mu at row i-1, columns k and k+1

    if (i0 >= 1) {
        const int i = i0 - 1;
        const long long c = (long long)i * NZ + kc;
        trr0 = ld(Fi, oTRR + c, kin);
        ttt0 = ld(Fi, oTTT + c, kin);
        tzz0 = ld(Fi, oTZZ + c, kin);
        trz0 = ld(Fi, oTRZ + c, kin);
        const long long m = mbase + (long long)i * S.model_ld;
        lam0 = ld(lam, m, kin);
        mu0 = ld(mu, m, kin);
        rho0 = ld(rho, m, kin);
    }

    for (int i = i0 - 1; i < i1; ++i) {
        const int ip = i + 1;
        // ---- load row ip
        float trr1 = 0.f, ttt1 = 0.f, tzz1 = 0.f, trz1 = 0.f, lam1 = 0.f, mu1 = 0.f, rho1 = 0.f,
              vro1 = 0.f;
        if (ip < NR) {
            const long long c = (long long)ip * NZ + kc;
            trr1 = ld(Fi, oTRR + c, kin);
            ttt1 = ld(Fi, oTTT + c, kin);
            tzz1 = ld(Fi, oTZZ + c, kin);
            trz1 = ld(Fi, oTRZ + c, kin);
            vro1 = ld(Fi, oVR + c, kin);
            const long long m = mbase + (long long)ip * S.model_ld;
            lam1 = ld(lam, m, kin);
            mu1 = ld(mu, m, kin);
            rho1 = ld(rho, m, kin);
        }
        // ---- v_r at R(ip), ip >= 1
        float vrn1 = 0.f;
        if (ip >= 1 && ip < NR) {
            const float trz1_km = sh_up(trz1);
            float Dr = (trr1 - trr0) * idr;
            float Dz = (trz1 - trz1_km) * idz;
            const bool st = own && ip < i1;
            if (ip >= nr) {  // PML memory A (radial, integer position)
                const long long q = oPR + 0LL * S.psir_len + ir(ip);
                const float psi = prt[NR + ip] * ld(Fi, q, kin) + prt[ip] * Dr;
                if (st) Fo[q] = psi;
                Dr += psi;
            }
            if (zp) {  // PML memory B (axial, integer position)
                const long long q = oPZ + 0LL * S.psiz_len + iz(ip);
                const float psi = b_zi * Fi[q] + a_zi * Dz;
                if (st) Fo[q] = psi;
                Dz += psi;
            }
            const float hoop = ((trr1 - ttt1) + (trr0 - ttt0)) * (0.5f / (ip * dr));
            const float bR = 2.0f / (rho0 + rho1);
            vrn1 = kin ? vro1 + dt * bR * (Dr + Dz + hoop) : 0.f;
        }
        // ---- v_z at Z(i), i >= 0
        float vzn0 = 0.f;
        const float tzz0_kp = sh_dn(tzz0);
        float rho0_kp = sh_dn(rho0);
        if (top) rho0_kp = rho0;
        if (i >= 0) {
            const long long c = (long long)i * NZ + kc;
            const float vzo = ld(Fi, oVZ + c, kin);
            float Dr = (trz1 - trz0) * idr;
            float Dz = (tzz0_kp - tzz0) * idz;
            const bool st = own && i >= i0;
            if (i >= nr) {  // C (radial, half position)
                const long long q = oPR + 1LL * S.psir_len + ir(i);
                const float psi = prt[3 * NR + i] * ld(Fi, q, kin) + prt[2 * NR + i] * Dr;
                if (st) Fo[q] = psi;
                Dr += psi;
            }
            if (zp) {  // D (axial, half position)
                const long long q = oPZ + 1LL * S.psiz_len + iz(i);
                const float psi = b_zh * Fi[q] + a_zh * Dz;
                if (st) Fo[q] = psi;
                Dz += psi;
            }
            const float hoop = (trz1 + trz0) * (0.5f / ((i + 0.5f) * dr));
            const float bZ = 2.0f / (rho0 + rho0_kp);
            vzn0 = kin ? vzo + dt * bZ * (Dr + Dz + hoop) : 0.f;
        }
        float mu0_kp = sh_dn(mu0);
        if (top) mu0_kp = mu0;
        const float vzn0_km = sh_up(vzn0);
        const float vrn0_kp = sh_dn(vrn0);
        if (i >= i0) {
            const long long c = (long long)i * NZ + kc;
            // ---- C node: normal stresses
            float err = (vrn1 - vrn0) * idr;
            const float ett = (vrn1 + vrn0) * (0.5f / ((i + 0.5f) * dr));
            float ezz = (vzn0 - vzn0_km) * idz;
            if (i >= nr) {  // E
                const long long q = oPR + 2LL * S.psir_len + ir(i);
                const float psi = prt[3 * NR + i] * ld(Fi, q, kin) + prt[2 * NR + i] * err;
                if (own) Fo[q] = psi;
                err += psi;
            }
            if (zp) {  // F
                const long long q = oPZ + 2LL * S.psiz_len + iz(i);
                const float psi = b_zi * Fi[q] + a_zi * ezz;
                if (own) Fo[q] = psi;
                ezz += psi;
            }
            const float tr = err + ett + ezz;
            float nrr = trr0 + dt * (lam0 * tr + 2.0f * mu0 * err);
            float ntt = ttt0 + dt * (lam0 * tr + 2.0f * mu0 * ett);
            float nzz = tzz0 + dt * (lam0 * tr + 2.0f * mu0 * ezz);
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
                    const long long q = oPZ + 3LL * S.psiz_len + iz(i);
                    const float psi = b_zh * Fi[q] + a_zh * ez;
                    if (own) Fo[q] = psi;
                    ez += psi;
                }
                if (i >= nr) {  // H
                    const long long q = oPR + 3LL * S.psir_len + ir(i);
                    const float psi = prt[NR + i] * ld(Fi, q, kin) + prt[i] * er;
                    if (own) Fo[q] = psi;
                    er += psi;
                }
                nrz = trz0 + dt * mu_harm(mum, mu0, mum_kp, mu0_kp) * (ez + er);
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
        // ---- rotate
        mum = mu0;
        mum_kp = mu0_kp;
        trr0 = trr1;
        ttt0 = ttt1;
        tzz0 = tzz1;
        trz0 = trz1;
        lam0 = lam1;
        mu0 = mu1;
        rho0 = rho1;
        vrn0 = vrn1;
        vznm = vzn0;
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
struct ARow {
    float trr, ttt, tzz, trz;     // adjoint stresses (residual injected)
    float lam, mu, rho, mu_kp;    // model at this row (mu_kp: column k+1, clamped)
    float Err, Ett, Ezz, Ez, Er;  // drivers of the transposed stress update
    float pTr, pRr, pTz, pZz, pG, pH;  // new Phi values (0 outside the PML)
};

__global__ void __launch_bounds__(512)
k_adj_step(const ShotDev* __restrict__ shots, const int4* __restrict__ work, int nwork, int n,
           const float* __restrict__ lam, const float* __restrict__ mu,
           const float* __restrict__ rho, const int* __restrict__ rec_k,
           const float* __restrict__ resid, const float* __restrict__ pml_r,
           const float* __restrict__ pml_z, const float* __restrict__ ain,
           float* __restrict__ aout, const float* __restrict__ hist, float* __restrict__ acc,
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
    const long long oPR = 6 * cells;
    const long long oPZ = oPR + 5LL * S.psir_len;
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

    // Load row ip of the adjoint state and model, compute the drivers of the
    // transposed stress update and the new Phi values.  mu_prev/_kp: row ip-1.
    auto load_row = [&](int ip, float mu_prev, float mu_prev_kp, bool store) -> ARow {
        ARow X{};
        X.pTr = X.pRr = X.pTz = X.pZz = X.pG = X.pH = 0.f;
        if (ip < 0 || ip >= NR) {
            X.mu_kp = 0.f;
            return X;
        }
        const long long c = (long long)ip * NZ + kc;
        X.trr = ld(Ai, oTRR + c, kin);
        X.ttt = ld(Ai, oTTT + c, kin);
        X.tzz = ld(Ai, oTZZ + c, kin);
        X.trz = (ip >= 1) ? ld(Ai, oTRZ + c, kin) : 0.f;
        if (ip == 0) {
            X.trr += inj;
            X.ttt += inj;
            X.tzz += inj;
        }
        const long long m = mbase + (long long)ip * S.model_ld;
        X.lam = ld(lam, m, kin);
        X.mu = ld(mu, m, kin);
        X.rho = ld(rho, m, kin);
        X.mu_kp = sh_dn(X.mu);
        if (top) X.mu_kp = X.mu;
        const float sa = X.trr + X.ttt + X.tzz;
        const float l = X.lam, mm2 = 2.0f * X.mu;
        X.Err = dt * (l * sa + mm2 * X.trr);
        X.Ett = dt * (l * sa + mm2 * X.ttt);
        X.Ezz = dt * (l * sa + mm2 * X.tzz);
        if (ip >= nr) {  // PhiT_r, PhiR_r at C (radial, half position)
            const float b = prt[3 * NR + ip], a = prt[2 * NR + ip];
            const long long qT = oPR + 2LL * S.psir_len + ir(ip);
            const long long qR = oPR + 3LL * S.psir_len + ir(ip);
            X.pTr = dt * sa + b * ld(Ai, qT, kin);
            X.pRr = dt * X.trr + b * ld(Ai, qR, kin);
            if (store) {
                Ao[qT] = X.pTr;
                Ao[qR] = X.pRr;
            }
            X.Err += a * (l * X.pTr + mm2 * X.pRr);
        }
        if (zp) {  // PhiT_z, PhiZ_z at C (axial, integer position)
            const long long qT = oPZ + 2LL * S.psiz_len + iz(ip);
            const long long qZ = oPZ + 3LL * S.psiz_len + iz(ip);
            X.pTz = dt * sa + b_zi * Ai[qT];
            X.pZz = dt * X.tzz + b_zi * Ai[qZ];
            if (store) {
                Ao[qT] = X.pTz;
                Ao[qZ] = X.pZz;
            }
            X.Ezz += a_zi * (l * X.pTz + mm2 * X.pZz);
        }
        X.Ez = 0.f;
        X.Er = 0.f;
        if (ip >= 1) {
            const float muS = mu_harm(mu_prev, X.mu, mu_prev_kp, X.mu_kp);
            const float s = dt * muS * X.trz;
            X.Ez = s;
            X.Er = s;
            if (zp) {  // PhiG at S (axial, half position)
                const long long q = oPZ + 4LL * S.psiz_len + iz(ip);
                X.pG = dt * X.trz + b_zh * Ai[q];
                if (store) Ao[q] = X.pG;
                X.Ez += a_zh * muS * X.pG;
            }
            if (ip >= nr) {  // PhiH at S (radial, integer position)
                const long long q = oPR + 4LL * S.psir_len + ir(ip);
                X.pH = dt * X.trz + prt[NR + ip] * ld(Ai, q, kin);
                if (store) Ao[q] = X.pH;
                X.Er += prt[ip] * muS * X.pH;
            }
        }
        if (!kin) {
            X.Err = X.Ett = X.Ezz = X.Ez = X.Er = 0.f;
        }
        return X;
    };

    ARow X0{};
    X0.pTr = X0.pRr = X0.pTz = X0.pZz = X0.pG = X0.pH = 0.f;
    if (i0 >= 1) {
        float mpp = 0.f, mpp_kp = 0.f;
        if (i0 >= 2) {
            mpp = ld(mu, mbase + (long long)(i0 - 2) * S.model_ld, kin);
            mpp_kp = sh_dn(mpp);
            if (top) mpp_kp = mpp;
        }
        X0 = load_row(i0 - 1, mpp, mpp_kp, false);
    }
    // R(i): [aDr, aDzR, hR]; Z(i-1) contribution to atrz(i): zm
    float R0_aDr = 0.f, R0_aDzR = 0.f, R0_hR = 0.f, zm = 0.f;
    float vrh0 = 0.f, vzhm = 0.f;
    if (i0 >= 1) vrh0 = ld(vrh, (long long)(i0 - 1) * NZ + kc, kin);

    for (int i = i0 - 1; i < i1; ++i) {
        const int ip = i + 1;
        const bool own_ip = own && ip >= i0 && ip < i1;
        const bool own_i = own && i >= i0;
        const ARow X1 = load_row(ip, X0.mu, X0.mu_kp, own_ip);
        // ---- R(ip): transposed stress update into avr, then transposed velocity update
        float R1_aDr = 0.f, R1_aDzR = 0.f, R1_hR = 0.f;
        const float Ez1_km = sh_up(X1.Ez);
        if (ip >= 1 && ip < NR) {
            const long long c = (long long)ip * NZ + kc;
            const float avr = ld(Ai, oVR + c, kin) + (X0.Err - X1.Err) * idr +
                              X0.Ett * (0.5f / ((ip - 0.5f) * dr)) +
                              X1.Ett * (0.5f / ((ip + 0.5f) * dr)) + (Ez1_km - X1.Ez) * idz;
            const float W = kin ? dt * (2.0f / (X0.rho + X1.rho)) * avr : 0.f;
            float aDr = W, aDz = W;
            if (ip >= nr) {  // A-bar
                const long long q = oPR + 0LL * S.psir_len + ir(ip);
                const float qv = ld(Ai, q, kin) + W;
                if (own_ip) Ao[q] = prt[NR + ip] * qv;
                aDr += prt[ip] * qv;
            }
            if (zp) {  // B-bar
                const long long q = oPZ + 0LL * S.psiz_len + iz(ip);
                const float qv = Ai[q] + W;
                if (own_ip) Ao[q] = b_zi * qv;
                aDz += a_zi * qv;
            }
            if (own_ip) Ao[oVR + c] = avr;
            R1_aDr = aDr;
            R1_aDzR = aDz;
            R1_hR = W * (0.5f / (ip * dr));
        }
        // ---- Z(i)
        float Z_aDrZ = 0.f, Z_WZ = 0.f, Z_aDzZ = 0.f;
        const float Ezz0_kp = sh_dn(X0.Ezz);
        float rho0_kp = sh_dn(X0.rho);
        if (top) rho0_kp = X0.rho;
        if (i >= 0) {
            const long long c = (long long)i * NZ + kc;
            const float avz = ld(Ai, oVZ + c, kin) + (X0.Ezz - Ezz0_kp) * idz +
                              (X0.Er - X1.Er) * idr;
            const float W = kin ? dt * (2.0f / (X0.rho + rho0_kp)) * avz : 0.f;
            float aDr = W, aDz = W;
            if (i >= nr) {  // C-bar (radial, half position)
                const long long q = oPR + 1LL * S.psir_len + ir(i);
                const float qv = ld(Ai, q, kin) + W;
                if (own_i) Ao[q] = prt[3 * NR + i] * qv;
                aDr += prt[2 * NR + i] * qv;
            }
            if (zp) {  // D-bar (axial, half position)
                const long long q = oPZ + 1LL * S.psiz_len + iz(i);
                const float qv = Ai[q] + W;
                if (own_i) Ao[q] = b_zh * qv;
                aDz += a_zh * qv;
            }
            if (own_i) Ao[oVZ + c] = avz;
            Z_aDrZ = aDr;
            Z_WZ = W;
            Z_aDzZ = aDz;
        }
        const float aDzZ_km = sh_up(Z_aDzZ);
        const float aDzR_kp = sh_dn(R0_aDzR);
        // ---- velocity history for the correlation at row i
        const float vrh1 = (ip < NR) ? ld(vrh, (long long)ip * NZ + kc, kin) : 0.f;
        const float vzh0 = (i >= 0) ? ld(vzh, (long long)i * NZ + kc, kin) : 0.f;
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
                nrz = X0.trz + (R0_aDzR - aDzR_kp) * idz - Z_aDrZ * idr + Z_WZ * (0.5f / rh) + zm;
            // Eq. 7-8: correlate the strain rates of v^{n+1/2} with dJ/dtau^{n+1}
            const float err = (vrh1 - vrh0) * idr;
            const float ett = (vrh1 + vrh0) * (0.5f / rh);
            const float ezz = (vzh0 - vzh0_km) * idz;
            const float sa = X0.trr + X0.ttt + X0.tzz;
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
            float dgs = 0.f;
            if (i >= 1) {
                const float ez = (vrh0_kp - vrh0) * idz;
                const float er = (vzh0 - vzhm) * idr;
                dgs = dt * (ez + er) * X0.trz;
                if (zp) dgs += a_zh * ez * X0.pG;
                if (i >= nr) dgs += prt[i] * er * X0.pH;
            }
            if (own) {
                Ao[oTRR + c] = nrr;
                Ao[oTTT + c] = ntt;
                Ao[oTZZ + c] = nzz;
                if (i >= 1) {
                    Ao[oTRZ + c] = nrz;
                    g_s[c] += dgs;
                }
                g_l[c] += dgl;
                g_m[c] += dgm;
                g_e[c] += dge;
            }
        }
        // ---- rotate
        zm = (i >= 0) ? Z_aDrZ * idr + Z_WZ * (0.5f / ((i + 0.5f) * dr)) : 0.f;
        X0 = X1;
        R0_aDr = R1_aDr;
        R0_aDzR = R1_aDzR;
        R0_hR = R1_hR;
        vrh0 = vrh1;
        vzhm = vzh0;
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

__global__ void __launch_bounds__(256)
k_sum_partials(int np, const double* __restrict__ part, double* __restrict__ out)
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
    if (threadIdx.x == 0) *out = sh[0];
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

__global__ void __launch_bounds__(256)
k_precond_apply(long long n, const uint8_t* __restrict__ mask, const float* __restrict__ illum,
                float eps, const float* __restrict__ part, int np, float* __restrict__ g_lam,
                float* __restrict__ g_mu)
{
    __shared__ float sh[256];
    const float emax = reduce_part_max(part, np, 0, sh);
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (!mask[i]) {
            g_lam[i] = 0.f;
            g_mu[i] = 0.f;
            continue;
        }
        const float p = 1.0f / (illum[i] + eps * emax);
        g_lam[i] *= p;
        g_mu[i] *= p;
    }
}

// part holds the maxima of |g_lam|, |g_mu|, |lam|, |mu| over mask cells.
__global__ void __launch_bounds__(256)
k_update_apply(long long n, const uint8_t* __restrict__ mask, float* __restrict__ lam,
               float* __restrict__ mu, const float* __restrict__ rho,
               const float* __restrict__ g_lam, const float* __restrict__ g_mu,
               const float* __restrict__ part, int np, float eta, float alpha_override,
               float vp_min, float vp_max, float vs_min, float vs_max,
               float* __restrict__ alpha_out)
{
    __shared__ float sh[256];
    float alpha = alpha_override;
    if (!(alpha > 0.f)) {
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
