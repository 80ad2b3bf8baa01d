// bhfwi_o4.hip -- fourth-order-in-space variant of the step of Eq. 2 and of
// its exact adjoint with the correlation of Eq. 7-8.
//
// The staggered grid, medium averaging, PML, source and receivers are those
// of the second-order kernels; every staggered difference and every two-point
// 1/r average becomes its four-point form
//   D f = [C1 (f(+1/2) - f(-1/2)) + C2 (f(+3/2) - f(-3/2))] / h,
//   I f =  G1 (f(+1/2) + f(-1/2)) + G2 (f(+3/2) + f(-3/2)),
// C1 = 9/8, C2 = -1/24, G1 = 9/16, G2 = -1/16.  Across the axis the fields
// are mirrored: normal stresses and v_z (half radial positions) are even,
// v_r and tau_rz (integer radial positions) odd and zero on the axis.
//
// One thread per cell and kernel; a cell reads its neighbours up to two rows
// away in r and z from global memory (L1/L2 serve the reuse).  The forward
// step is two kernels (velocities, then stresses).  The adjoint is three, the
// transposes in gather form: A turns the adjoint stresses into the drivers of
// the transposed stress update (and correlates them with the stored velocity
// strain rates), B gathers the drivers into the adjoint velocities and forms
// the products of the transposed velocity update, C gathers those into the
// adjoint stresses.  A gather that the forward stencil reached through the
// mirror is folded back: the gather at the mirrored (logical, negative) row is
// added to its image with the field's parity.
#pragma once
#include "bhfwi_internal.h"

namespace bhfwi {
namespace o4 {

constexpr float C1 = 9.0f / 8.0f, C2 = -1.0f / 24.0f, G1 = 9.0f / 16.0f, G2 = -1.0f / 16.0f;

// The shot and cell of a flat thread index over the packed per-cell planes
// (shots in increasing cell_off); false for the alignment gaps.
__device__ inline bool locate(const ShotDev* __restrict__ shots, int nshot, long long t, int* s,
                              int* i, int* k)
{
    int lo = 0, hi = nshot - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (shots[mid].cell_off <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    const ShotDev& S = shots[lo];
    const long long c = t - S.cell_off;
    if (c < 0 || c >= (long long)S.NR * S.NZ) return false;
    *s = lo;
    *i = (int)(c / S.NZ);
    *k = (int)(c % S.NZ);
    return true;
}

// Field values with the boundary rules: zero outside [0, NZ) and beyond the
// outer radius; mirrored across the axis (even at half radial positions, odd
// and zero on the axis at integer ones).
struct Grid {
    int NR, NZ;
    __device__ float even(const float* __restrict__ p, int i, int k) const
    {
        if (k < 0 || k >= NZ) return 0.f;
        if (i < 0) i = -1 - i;
        if (i >= NR) return 0.f;
        return p[(long long)i * NZ + k];
    }
    __device__ float odd(const float* __restrict__ p, int i, int k) const
    {
        if (k < 0 || k >= NZ) return 0.f;
        float sg = 1.f;
        if (i < 0) {
            i = -i;
            sg = -1.f;
        }
        if (i == 0 || i >= NR) return 0.f;
        return sg * p[(long long)i * NZ + k];
    }
    // a per-node product (zero outside the grid, no mirror: the fold does it)
    __device__ float at(const float* __restrict__ p, int i, int k) const
    {
        if (k < 0 || k >= NZ || i < 0 || i >= NR) return 0.f;
        return p[(long long)i * NZ + k];
    }
};

__device__ inline float harm4(float a, float b, float c, float d)
{
    return (a > 0.f && b > 0.f && c > 0.f && d > 0.f)
               ? 4.0f / (1.0f / a + 1.0f / b + 1.0f / c + 1.0f / d)
               : 0.0f;
}

// ---------------------------------------------------------------------------
// Forward.  State block as in the second-order kernels: 6 fields, then 4
// radial PML strips [A, C, E, H] of pr*NZ, then 4 axial strips [B, D, F, G]
// of NR*2pz.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_fwd4_vel(const ShotDev* __restrict__ shots, int nshot, long long ncell, int n,
           const float* __restrict__ rho, const float* __restrict__ pml_r,
           const float* __restrict__ pml_z, const float* __restrict__ sin,
           float* __restrict__ sout, float* __restrict__ hist, long long cells_total)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int s, i, k;
    if (t >= ncell || !locate(shots, nshot, t, &s, &i, &k)) return;
    const ShotDev& S = shots[s];
    if (n >= S.nt) return;
    const int NR = S.NR, NZ = S.NZ, nr = S.nr, pz = S.pz;
    const Grid g{NR, NZ};
    const long long cells = (long long)NR * NZ, c = (long long)i * NZ + k;
    const float* __restrict__ Fi = sin + S.fst_off;
    float* __restrict__ Fo = sout + S.fst_off;
    const float *vr = Fi, *vz = Fi + cells, *trr = Fi + 2 * cells, *ttt = Fi + 3 * cells,
                *tzz = Fi + 4 * cells, *trz = Fi + 5 * cells;
    const long long LR = S.psir_len, LZ = S.psiz_len, oPR = 6 * cells, oPZ = oPR + 4 * LR;
    const float* __restrict__ prt = pml_r + S.pml_r_off;
    const float* __restrict__ pzt = pml_z + S.pml_z_off;
    const bool zp = k < pz || k >= NZ - pz;
    const int kk = zp ? (k < pz ? k : k - (NZ - 2 * pz)) : 0;
    const float dt = S.dt, idr = S.inv_dr, idz = S.inv_dz, dr = S.dr;
    const long long m = S.model_off + (long long)i * S.model_ld + k;

    // ---- v_r at R(i, k), i >= 1
    float vrn = 0.f;
    if (i >= 1) {
        float Dr = (C1 * (g.even(trr, i, k) - g.even(trr, i - 1, k)) +
                    C2 * (g.even(trr, i + 1, k) - g.even(trr, i - 2, k))) * idr;
        float Dz = (C1 * (g.odd(trz, i, k) - g.odd(trz, i, k - 1)) +
                    C2 * (g.odd(trz, i, k + 1) - g.odd(trz, i, k - 2))) * idz;
        auto d = [&](int ii) { return g.even(trr, ii, k) - g.even(ttt, ii, k); };
        const float hoop = (G1 * (d(i) + d(i - 1)) + G2 * (d(i + 1) + d(i - 2))) / (i * dr);
        if (i >= nr) {  // A
            const long long q = oPR + (long long)(i - nr) * NZ + k;
            const float psi = prt[NR + i] * Fi[q] + prt[i] * Dr;
            Fo[q] = psi;
            Dr += psi;
        }
        if (zp) {  // B
            const long long q = oPZ + (long long)i * (2 * pz) + kk;
            const float psi = pzt[NZ + k] * Fi[q] + pzt[k] * Dz;
            Fo[q] = psi;
            Dz += psi;
        }
        const float bR = 2.0f / (rho[m - S.model_ld] + rho[m]);
        vrn = vr[c] + dt * bR * (Dr + Dz + hoop);
        Fo[c] = vrn;
    }
    // ---- v_z at Z(i, k)
    float Dr = (C1 * (g.odd(trz, i + 1, k) - g.odd(trz, i, k)) +
                C2 * (g.odd(trz, i + 2, k) - g.odd(trz, i - 1, k))) * idr;
    float Dz = (C1 * (g.even(tzz, i, k + 1) - g.even(tzz, i, k)) +
                C2 * (g.even(tzz, i, k + 2) - g.even(tzz, i, k - 1))) * idz;
    const float hoop = (G1 * (g.odd(trz, i + 1, k) + g.odd(trz, i, k)) +
                        G2 * (g.odd(trz, i + 2, k) + g.odd(trz, i - 1, k))) / ((i + 0.5f) * dr);
    if (i >= nr) {  // C
        const long long q = oPR + LR + (long long)(i - nr) * NZ + k;
        const float psi = prt[3 * NR + i] * Fi[q] + prt[2 * NR + i] * Dr;
        Fo[q] = psi;
        Dr += psi;
    }
    if (zp) {  // D
        const long long q = oPZ + LZ + (long long)i * (2 * pz) + kk;
        const float psi = pzt[3 * NZ + k] * Fi[q] + pzt[2 * NZ + k] * Dz;
        Fo[q] = psi;
        Dz += psi;
    }
    const int k1 = k + 1 < NZ ? k + 1 : NZ - 1;
    const float bZ = 2.0f / (rho[m] + rho[m - k + k1]);
    const float vzn = vz[c] + dt * bZ * (Dr + Dz + hoop);
    Fo[cells + c] = vzn;
    if (hist) {
        hist[S.cell_off + c] = vrn;
        hist[cells_total + S.cell_off + c] = vzn;
    }
}

__global__ void __launch_bounds__(256)
k_fwd4_str(const ShotDev* __restrict__ shots, int nshot, long long ncell, int n,
           const float* __restrict__ lam, const float* __restrict__ mu,
           const float* __restrict__ wavelet, const int* __restrict__ rec_k,
           const float* __restrict__ pml_r, const float* __restrict__ pml_z,
           const float* __restrict__ sin, float* __restrict__ sout, float* __restrict__ traces)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int s, i, k;
    if (t >= ncell || !locate(shots, nshot, t, &s, &i, &k)) return;
    const ShotDev& S = shots[s];
    if (n >= S.nt) return;
    const int NR = S.NR, NZ = S.NZ, nr = S.nr, pz = S.pz;
    const Grid g{NR, NZ};
    const long long cells = (long long)NR * NZ, c = (long long)i * NZ + k;
    const float* __restrict__ Fi = sin + S.fst_off;
    float* __restrict__ Fo = sout + S.fst_off;
    const float *vr = Fo, *vz = Fo + cells;  // the new velocities
    const long long LR = S.psir_len, LZ = S.psiz_len, oPR = 6 * cells, oPZ = oPR + 4 * LR;
    const float* __restrict__ prt = pml_r + S.pml_r_off;
    const float* __restrict__ pzt = pml_z + S.pml_z_off;
    const bool zp = k < pz || k >= NZ - pz;
    const int kk = zp ? (k < pz ? k : k - (NZ - 2 * pz)) : 0;
    const float dt = S.dt, idr = S.inv_dr, idz = S.inv_dz, dr = S.dr;
    const long long m = S.model_off + (long long)i * S.model_ld + k;

    // ---- normal stresses at C(i, k)
    float err = (C1 * (g.odd(vr, i + 1, k) - g.odd(vr, i, k)) +
                 C2 * (g.odd(vr, i + 2, k) - g.odd(vr, i - 1, k))) * idr;
    const float ett = (G1 * (g.odd(vr, i + 1, k) + g.odd(vr, i, k)) +
                       G2 * (g.odd(vr, i + 2, k) + g.odd(vr, i - 1, k))) / ((i + 0.5f) * dr);
    float ezz = (C1 * (g.even(vz, i, k) - g.even(vz, i, k - 1)) +
                 C2 * (g.even(vz, i, k + 1) - g.even(vz, i, k - 2))) * idz;
    if (i >= nr) {  // E
        const long long q = oPR + 2 * LR + (long long)(i - nr) * NZ + k;
        const float psi = prt[3 * NR + i] * Fi[q] + prt[2 * NR + i] * err;
        Fo[q] = psi;
        err += psi;
    }
    if (zp) {  // F
        const long long q = oPZ + 2 * LZ + (long long)i * (2 * pz) + kk;
        const float psi = pzt[NZ + k] * Fi[q] + pzt[k] * ezz;
        Fo[q] = psi;
        ezz += psi;
    }
    const float l = lam[m], u = mu[m];
    const float tr = err + ett + ezz;
    float nrr = Fi[2 * cells + c] + dt * (l * tr + 2.0f * u * err);
    float ntt = Fi[3 * cells + c] + dt * (l * tr + 2.0f * u * ett);
    float nzz = Fi[4 * cells + c] + dt * (l * tr + 2.0f * u * ezz);
    if (i == 0 && k == S.src_k) {
        const float sv = S.src_scale * wavelet[S.wave_off + n];
        nrr += sv;
        ntt += sv;
        nzz += sv;
    }
    Fo[2 * cells + c] = nrr;
    Fo[3 * cells + c] = ntt;
    Fo[4 * cells + c] = nzz;
    if (i == 0 && traces)
        for (int j = 0; j < S.nrec; ++j)
            if (rec_k[S.rec_off + j] == k)
                traces[S.trace_off + (long long)j * S.nt + n] = (nrr + ntt + nzz) * (1.0f / 3.0f);
    // ---- tau_rz at S(i, k), i >= 1
    if (i >= 1) {
        float ez = (C1 * (g.odd(vr, i, k + 1) - g.odd(vr, i, k)) +
                    C2 * (g.odd(vr, i, k + 2) - g.odd(vr, i, k - 1))) * idz;
        float er = (C1 * (g.even(vz, i, k) - g.even(vz, i - 1, k)) +
                    C2 * (g.even(vz, i + 1, k) - g.even(vz, i - 2, k))) * idr;
        if (zp) {  // G
            const long long q = oPZ + 3 * LZ + (long long)i * (2 * pz) + kk;
            const float psi = pzt[3 * NZ + k] * Fi[q] + pzt[2 * NZ + k] * ez;
            Fo[q] = psi;
            ez += psi;
        }
        if (i >= nr) {  // H
            const long long q = oPR + 3 * LR + (long long)(i - nr) * NZ + k;
            const float psi = prt[NR + i] * Fi[q] + prt[i] * er;
            Fo[q] = psi;
            er += psi;
        }
        const int k1 = k + 1 < NZ ? k + 1 : NZ - 1;
        const long long mm = m - S.model_ld;
        const float muS = harm4(mu[mm], u, mu[mm - k + k1], mu[m - k + k1]);
        Fo[5 * cells + c] = Fi[5 * cells + c] + dt * muS * (ez + er);
    }
}

// ---------------------------------------------------------------------------
// Adjoint.  Adjoint state block as in the second-order kernels: 6 fields, 5
// radial strips [A-bar, C-bar, PhiT_r, PhiR_r, PhiH], 5 axial strips [B-bar,
// D-bar, PhiT_z, PhiZ_z, PhiG].  Scratch planes (cells_total each): drivers
// [Err, Ett, Ezz, Ez, Er], products [UR, HR, DZR, ZR, ZH, DZZ].
// ---------------------------------------------------------------------------
enum { D_ERR = 0, D_ETT, D_EZZ, D_EZ, D_ER, P_UR, P_HR, P_DZR, P_ZR, P_ZH, P_DZZ, N_SCR };

__global__ void __launch_bounds__(256)
k_adj4_drivers(const ShotDev* __restrict__ shots, int nshot, long long ncell, int n,
               const float* __restrict__ lam, const float* __restrict__ mu,
               const int* __restrict__ rec_k, const float* __restrict__ resid,
               const float* __restrict__ pml_r, const float* __restrict__ pml_z,
               const float* __restrict__ ain, float* __restrict__ aout,
               const float* __restrict__ hist, float* __restrict__ scr,
               float* __restrict__ acc, long long cells_total)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int s, i, k;
    if (t >= ncell || !locate(shots, nshot, t, &s, &i, &k)) return;
    const ShotDev& S = shots[s];
    if (n >= S.nt) return;
    const int NR = S.NR, NZ = S.NZ, nr = S.nr, pz = S.pz;
    const Grid g{NR, NZ};
    const long long cells = (long long)NR * NZ, c = (long long)i * NZ + k;
    const float* __restrict__ Ai = ain + S.ast_off;
    float* __restrict__ Ao = aout + S.ast_off;
    const long long LR = S.psir_len, LZ = S.psiz_len, oPR = 6 * cells, oPZ = oPR + 5 * LR;
    const float* __restrict__ prt = pml_r + S.pml_r_off;
    const float* __restrict__ pzt = pml_z + S.pml_z_off;
    const bool zp = k < pz || k >= NZ - pz;
    const int kk = zp ? (k < pz ? k : k - (NZ - 2 * pz)) : 0;
    const float dt = S.dt, idr = S.inv_dr, idz = S.inv_dz, dr = S.dr;
    const long long m = S.model_off + (long long)i * S.model_ld + k;
    float* __restrict__ sc = scr + S.cell_off + c;

    // ---- C node: residual, drivers, Phi recursions
    float trr = Ai[2 * cells + c], ttt = Ai[3 * cells + c], tzz = Ai[4 * cells + c];
    if (i == 0) {
        float inj = 0.f;
        for (int j = 0; j < S.nrec; ++j)
            if (rec_k[S.rec_off + j] == k) inj += resid[S.trace_off + (long long)j * S.nt + n];
        inj *= (1.0f / 3.0f);
        trr += inj;
        ttt += inj;
        tzz += inj;
    }
    Ao[2 * cells + c] = trr;
    Ao[3 * cells + c] = ttt;
    Ao[4 * cells + c] = tzz;
    const float l = lam[m], u = mu[m], sa = trr + ttt + tzz;
    float Err = dt * (l * sa + 2.0f * u * trr);
    const float Ett = dt * (l * sa + 2.0f * u * ttt);
    float Ezz = dt * (l * sa + 2.0f * u * tzz);
    float pTr = 0.f, pRr = 0.f, pTz = 0.f, pZz = 0.f, a_rh = 0.f;
    if (i >= nr) {
        const long long q = oPR + (long long)(i - nr) * NZ + k;
        const float b = prt[3 * NR + i];
        a_rh = prt[2 * NR + i];
        pTr = dt * sa + b * Ai[q + 2 * LR];
        pRr = dt * trr + b * Ai[q + 3 * LR];
        Ao[q + 2 * LR] = pTr;
        Ao[q + 3 * LR] = pRr;
        Err += a_rh * (l * pTr + 2.0f * u * pRr);
    }
    const float a_zi = zp ? pzt[k] : 0.f;
    if (zp) {
        const long long q = oPZ + (long long)i * (2 * pz) + kk;
        const float b = pzt[NZ + k];
        pTz = dt * sa + b * Ai[q + 2 * LZ];
        pZz = dt * tzz + b * Ai[q + 3 * LZ];
        Ao[q + 2 * LZ] = pTz;
        Ao[q + 3 * LZ] = pZz;
        Ezz += a_zi * (l * pTz + 2.0f * u * pZz);
    }
    // ---- S node (i >= 1)
    float trz = 0.f, Ez = 0.f, Er = 0.f, pG = 0.f, pH = 0.f, a_zh = 0.f, a_ri = 0.f;
    if (i >= 1) {
        trz = Ai[5 * cells + c];
        const int k1 = k + 1 < NZ ? k + 1 : NZ - 1;
        const long long mm = m - S.model_ld;
        const float muS = harm4(mu[mm], u, mu[mm - k + k1], mu[m - k + k1]);
        Ez = Er = dt * muS * trz;
        if (zp) {
            const long long q = oPZ + 4 * LZ + (long long)i * (2 * pz) + kk;
            a_zh = pzt[2 * NZ + k];
            pG = dt * trz + pzt[3 * NZ + k] * Ai[q];
            Ao[q] = pG;
            Ez += a_zh * muS * pG;
        }
        if (i >= nr) {
            const long long q = oPR + 4 * LR + (long long)(i - nr) * NZ + k;
            a_ri = prt[i];
            pH = dt * trz + prt[NR + i] * Ai[q];
            Ao[q] = pH;
            Er += a_ri * muS * pH;
        }
    }
    Ao[5 * cells + c] = trz;
    sc[D_ERR * cells_total] = Err;
    sc[D_ETT * cells_total] = Ett;
    sc[D_EZZ * cells_total] = Ezz;
    sc[D_EZ * cells_total] = Ez;
    sc[D_ER * cells_total] = Er;

    // ---- Eq. 7-8 with the strain rates of the stored v^{n+1/2}
    const float* vrh = hist + S.cell_off;
    const float* vzh = hist + cells_total + S.cell_off;
    const float vr0 = g.odd(vrh, i, k), vr1 = g.odd(vrh, i + 1, k);
    const float err = (C1 * (vr1 - vr0) + C2 * (g.odd(vrh, i + 2, k) - g.odd(vrh, i - 1, k))) * idr;
    const float ett = (G1 * (vr1 + vr0) + G2 * (g.odd(vrh, i + 2, k) + g.odd(vrh, i - 1, k))) /
                      ((i + 0.5f) * dr);
    const float vz0 = g.even(vzh, i, k), vzm = g.even(vzh, i, k - 1);
    const float ezz = (C1 * (vz0 - vzm) + C2 * (g.even(vzh, i, k + 1) - g.even(vzh, i, k - 2))) * idz;
    float dgl = dt * (err + ett + ezz) * sa + a_rh * err * pTr + a_zi * ezz * pTz;
    float dgm = 2.0f * dt * (err * trr + ett * ttt + ezz * tzz) +
                2.0f * (a_rh * err * pRr + a_zi * ezz * pZz);
    const float ur = 0.5f * (vr0 + vr1), uz = 0.5f * (vzm + vz0);
    float* ga = acc + S.cell_off + c;
    ga[0] += dgl;
    ga[cells_total] += dgm;
    ga[3 * cells_total] += dt * (ur * ur + uz * uz);
    if (i >= 1) {
        const float ez = (C1 * (g.odd(vrh, i, k + 1) - vr0) +
                          C2 * (g.odd(vrh, i, k + 2) - g.odd(vrh, i, k - 1))) * idz;
        const float er = (C1 * (vz0 - g.even(vzh, i - 1, k)) +
                          C2 * (g.even(vzh, i + 1, k) - g.even(vzh, i - 2, k))) * idr;
        ga[2 * cells_total] += dt * (ez + er) * trz + a_zh * ez * pG + a_ri * er * pH;
    }
}

// Transposed gathers.  P holds per-node values of one shot (rows of NZ);
// "lo" rows are the output rows whose forward stencil read the field at rows
// j - 1 and j (+ C2 at j + 1, j - 2); "hi" rows read j and j + 1.
//   gat_lo: sum_i dcoef(i, j) P[i] for the difference evaluated at integer
//           nodes from half-position inputs (F1, F4, Z1 patterns),
//   gat_hi: the same for half-position outputs from integer inputs (F2, F3,
//           Z2 patterns).
struct Gather {
    Grid g;
    // D^T of an integer-output stencil (out i reads in i-1, i; i-2, i+1), at
    // input row j along r
    __device__ float Dlo_r(const float* P, int j, int k) const
    {
        return C1 * (g.at(P, j, k) - g.at(P, j + 1, k)) + C2 * (g.at(P, j - 1, k) - g.at(P, j + 2, k));
    }
    __device__ float Ilo_r(const float* P, int j, int k) const
    {
        return G1 * (g.at(P, j, k) + g.at(P, j + 1, k)) + G2 * (g.at(P, j - 1, k) + g.at(P, j + 2, k));
    }
    // D^T of a half-output stencil (out i reads in i, i+1; i-1, i+2)
    __device__ float Dhi_r(const float* P, int j, int k) const
    {
        return C1 * (g.at(P, j - 1, k) - g.at(P, j, k)) + C2 * (g.at(P, j - 2, k) - g.at(P, j + 1, k));
    }
    __device__ float Ihi_r(const float* P, int j, int k) const
    {
        return G1 * (g.at(P, j - 1, k) + g.at(P, j, k)) + G2 * (g.at(P, j - 2, k) + g.at(P, j + 1, k));
    }
    __device__ float Dlo_z(const float* P, int i, int j) const
    {
        return C1 * (g.at(P, i, j) - g.at(P, i, j + 1)) + C2 * (g.at(P, i, j - 1) - g.at(P, i, j + 2));
    }
    __device__ float Dhi_z(const float* P, int i, int j) const
    {
        return C1 * (g.at(P, i, j - 1) - g.at(P, i, j)) + C2 * (g.at(P, i, j - 2) - g.at(P, i, j + 1));
    }
    // folded radial gathers: an even (half-position) input row j in {0, 1}
    // also receives its mirror row -1 - j; an odd (integer) input row 1 the
    // negated gather of row -1
    __device__ float Dlo_r_even(const float* P, int j, int k) const
    {
        return Dlo_r(P, j, k) + (j <= 1 ? Dlo_r(P, -1 - j, k) : 0.f);
    }
    __device__ float Ilo_r_even(const float* P, int j, int k) const
    {
        return Ilo_r(P, j, k) + (j <= 1 ? Ilo_r(P, -1 - j, k) : 0.f);
    }
    __device__ float Dhi_r_odd(const float* P, int j, int k) const
    {
        return Dhi_r(P, j, k) - (j == 1 ? Dhi_r(P, -1, k) : 0.f);
    }
    __device__ float Ihi_r_odd(const float* P, int j, int k) const
    {
        return Ihi_r(P, j, k) - (j == 1 ? Ihi_r(P, -1, k) : 0.f);
    }
};

__global__ void __launch_bounds__(256)
k_adj4_velocity(const ShotDev* __restrict__ shots, int nshot, long long ncell, int n,
                const float* __restrict__ rho, const float* __restrict__ pml_r,
                const float* __restrict__ pml_z, const float* __restrict__ ain,
                float* __restrict__ aout, float* __restrict__ scr, long long cells_total)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int s, i, k;
    if (t >= ncell || !locate(shots, nshot, t, &s, &i, &k)) return;
    const ShotDev& S = shots[s];
    if (n >= S.nt) return;
    const int NR = S.NR, NZ = S.NZ, nr = S.nr, pz = S.pz;
    const Gather G{{NR, NZ}};
    const long long cells = (long long)NR * NZ, c = (long long)i * NZ + k;
    const float* __restrict__ Ai = ain + S.ast_off;
    float* __restrict__ Ao = aout + S.ast_off;
    const long long LR = S.psir_len, LZ = S.psiz_len, oPR = 6 * cells, oPZ = oPR + 5 * LR;
    const float* __restrict__ prt = pml_r + S.pml_r_off;
    const float* __restrict__ pzt = pml_z + S.pml_z_off;
    const bool zp = k < pz || k >= NZ - pz;
    const int kk = zp ? (k < pz ? k : k - (NZ - 2 * pz)) : 0;
    const float dt = S.dt, idr = S.inv_dr, idz = S.inv_dz, dr = S.dr;
    const long long m = S.model_off + (long long)i * S.model_ld + k;
    float* __restrict__ base = scr + S.cell_off;
    const float* Err = base + D_ERR * cells_total;
    const float* Ett = base + D_ETT * cells_total;
    const float* Ezz = base + D_EZZ * cells_total;
    const float* Ez = base + D_EZ * cells_total;
    const float* Er = base + D_ER * cells_total;

    // ---- a_v_r at R(i, k), i >= 1: the stress update read v_r through e_rr
    // (C, half output), e_tt (C, I / r) and e_z (S, axial half output)
    float UR = 0.f, HR = 0.f, DZR = 0.f;
    if (i >= 1) {
        // e_tt carries 1/r_C: gather Ett / r_C
        auto q = [&](int ii) { return ii >= 0 && ii < NR ? 1.0f / ((ii + 0.5f) * dr) : 0.f; };
        float it = G1 * (G.g.at(Ett, i - 1, k) * q(i - 1) + G.g.at(Ett, i, k) * q(i)) +
                   G2 * (G.g.at(Ett, i - 2, k) * q(i - 2) + G.g.at(Ett, i + 1, k) * q(i + 1));
        if (i == 1) it -= G2 * G.g.at(Ett, 0, k) * q(0);  // mirror of row -1
        const float dar = G.Dhi_r_odd(Err, i, k) * idr + it + G.Dhi_z(Ez, i, k) * idz;
        const float avr = Ai[c] + dar;
        Ao[c] = avr;
        const float W1 = dt * 2.0f / (rho[m - S.model_ld] + rho[m]) * avr;
        float aDr = W1, aDz = W1;
        if (i >= nr) {  // A-bar
            const long long qq = oPR + (long long)(i - nr) * NZ + k;
            const float v = Ai[qq] + W1;
            Ao[qq] = prt[NR + i] * v;
            aDr += prt[i] * v;
        }
        if (zp) {  // B-bar
            const long long qq = oPZ + (long long)i * (2 * pz) + kk;
            const float v = Ai[qq] + W1;
            Ao[qq] = pzt[NZ + k] * v;
            aDz += pzt[k] * v;
        }
        UR = aDr;
        HR = W1 / (i * dr);
        DZR = aDz;
    }
    // ---- a_v_z at Z(i, k): read through e_zz (C, axial integer output) and
    // e_r (S, radial integer output)
    const float daz = G.Dlo_z(Ezz, i, k) * idz + G.Dlo_r_even(Er, i, k) * idr;
    const float avz = Ai[cells + c] + daz;
    Ao[cells + c] = avz;
    const int k1 = k + 1 < NZ ? k + 1 : NZ - 1;
    const float W2 = dt * 2.0f / (rho[m] + rho[m - k + k1]) * avz;
    float aDr = W2, aDz = W2;
    if (i >= nr) {  // C-bar
        const long long qq = oPR + LR + (long long)(i - nr) * NZ + k;
        const float v = Ai[qq] + W2;
        Ao[qq] = prt[3 * NR + i] * v;
        aDr += prt[2 * NR + i] * v;
    }
    if (zp) {  // D-bar
        const long long qq = oPZ + LZ + (long long)i * (2 * pz) + kk;
        const float v = Ai[qq] + W2;
        Ao[qq] = pzt[3 * NZ + k] * v;
        aDz += pzt[2 * NZ + k] * v;
    }
    float* sc = base + c;
    sc[P_UR * cells_total] = UR;
    sc[P_HR * cells_total] = HR;
    sc[P_DZR * cells_total] = DZR;
    sc[P_ZR * cells_total] = aDr;
    sc[P_ZH * cells_total] = W2 / ((i + 0.5f) * dr);
    sc[P_DZZ * cells_total] = aDz;
}

__global__ void __launch_bounds__(256)
k_adj4_stress(const ShotDev* __restrict__ shots, int nshot, long long ncell, int n,
              float* __restrict__ aout, const float* __restrict__ scr, long long cells_total)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int s, i, k;
    if (t >= ncell || !locate(shots, nshot, t, &s, &i, &k)) return;
    const ShotDev& S = shots[s];
    if (n >= S.nt) return;
    const int NR = S.NR, NZ = S.NZ;
    const Gather G{{NR, NZ}};
    const long long cells = (long long)NR * NZ, c = (long long)i * NZ + k;
    float* __restrict__ Ao = aout + S.ast_off;
    const float idr = S.inv_dr, idz = S.inv_dz;
    const float* base = scr + S.cell_off;
    const float* UR = base + P_UR * cells_total;
    const float* HR = base + P_HR * cells_total;
    const float* DZR = base + P_DZR * cells_total;
    const float* ZR = base + P_ZR * cells_total;
    const float* ZH = base + P_ZH * cells_total;
    const float* DZZ = base + P_DZZ * cells_total;
    // C node: the velocity update read tau_rr (D and I at R nodes, integer
    // outputs from half inputs), tau_tt (-I at R nodes), tau_zz (Z nodes, axial
    // half outputs)
    const float h = G.Ilo_r_even(HR, i, k);
    Ao[2 * cells + c] += G.Dlo_r_even(UR, i, k) * idr + h;
    Ao[3 * cells + c] -= h;
    Ao[4 * cells + c] += G.Dhi_z(DZZ, i, k) * idz;
    // S node: tau_rz read by v_r (axial integer output from half inputs) and by
    // v_z (radial half outputs from integer inputs, D and I)
    if (i >= 1)
        Ao[5 * cells + c] += G.Dlo_z(DZR, i, k) * idz + G.Dhi_r_odd(ZR, i, k) * idr +
                             G.Ihi_r_odd(ZH, i, k);
}

}  // namespace o4
}  // namespace bhfwi
