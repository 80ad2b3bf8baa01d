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
// v_r and tau_rz (integer radial positions) odd and zero on the axis, and the
// on-axis source is normalised by the axis cell's weight (AXIS_SRC).
//
// One kernel per step and direction, on tiles of TK = 64 axial by TI = 12
// radial cells with one thread per owned cell (768 threads; taller tiles were
// measured slower).  The stages of
// a step stay in LDS with halo recomputation: the forward stages the stresses
// on the tile plus four cells, forms the new velocities on the tile plus two
// (the halo cells' values are recomputed by every tile that needs them) and
// updates the stresses of the owned cells.  The adjoint, in gather form,
// forms the drivers of the transposed stress update on the tile plus four,
// the adjoint velocities and the products of the transposed velocity update
// on the tile plus two, and gathers those into the adjoint stresses of the
// owned cells, where it also correlates them with the stored velocity strain
// rates (Eq. 7-8).  A gather that the forward stencil reached through the
// mirror is folded back: the gather at the mirrored (logical, negative) row is
// added to its image with the field's parity.
//
// A single step per launch leaves little arithmetic to hide memory latency
// behind, so each thread issues every load that does not depend on the LDS
// stages of the step before the first barrier: for its owned cell and for at
// most one halo cell of each region, the stresses (forward) or the adjoint
// point (adjoint) of the D-region, the old velocities and buoyancies of the
// P-region, the moduli, and the gradient accumulators.
#pragma once
#include "bhfwi_internal.h"

namespace bhfwi {
namespace o4 {

constexpr float C1 = 9.0f / 8.0f, C2 = -1.0f / 24.0f, G1 = 9.0f / 16.0f, G2 = -1.0f / 16.0f;

// Source normalisation on the axis.  Mirrored across the axis, the four-point
// radial divergence conserves the flux sum_i w_i h r_{i+1/2} div_i only for
// near-axis cell weights w_i = 1 - z^i / (7 + sqrt 42), z = 13 - 2 sqrt 42
// (the bounded solution of C1 (w_{j-1} - w_j) + C2 (w_{j-2} - w_{j+1}) = 0
// that also cancels the image term C2 F_{-1} = C2 F_1 at the first node).
// The on-axis cell weighs w_0 = sqrt(6/7) of its volume, so the source is
// injected divided by that weight: sqrt(7/6).
constexpr float AXIS_SRC = 1.0801234497346435f;

constexpr int TK = 64, TI = 12;
// P-region: the tile plus two cells; D-region: the tile plus four
constexpr int PW = TK + 4, PH = TI + 4, PN = PW * PH;
constexpr int DW = TK + 8, DH = TI + 8, DN = DW * DH;

// The shot and first cell (i0, k0) of tile b: tile_start[s] is the first
// tile of shot s (tiles of a shot radial-major, ceil(NZ / TK) per row band).
__device__ inline bool tile_of(const ShotDev* __restrict__ shots,
                               const int* __restrict__ tile_start, int nshot, int b, int* s,
                               int* i0, int* k0)
{
    int lo = 0, hi = nshot - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tile_start[mid] <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int local = b - tile_start[lo];
    const ShotDev& S = shots[lo];
    const int nk = (S.NZ + TK - 1) / TK;
    if (local >= nk * ((S.NR + TI - 1) / TI)) return false;
    *s = lo;
    *i0 = (local / nk) * TI;
    *k0 = (local % nk) * TK;
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
};

// An LDS region read at grid cell (i, k), which must lie inside it; at()
// reads zero at negative rows (per-node products have no mirror).
struct View {
    const float* L;
    int ilo, klo, w;
    __device__ float operator()(int i, int k) const { return L[(i - ilo) * w + (k - klo)]; }
    __device__ float at(int i, int k) const { return i < 0 ? 0.f : (*this)(i, k); }
};

__device__ inline float harm4(float a, float b, float c, float d)
{
    return (a > 0.f && b > 0.f && c > 0.f && d > 0.f)
               ? 4.0f / (1.0f / a + 1.0f / b + 1.0f / c + 1.0f / d)
               : 0.0f;
}


// The tile of this workgroup and the shot it belongs to; threads past the
// grid still take part in the staging.
#define O4_PROLOGUE                                                                   \
    int s, i0, k0;                                                                    \
    if (!tile_of(shots, tile_start, nshot, (int)blockIdx.x, &s, &i0, &k0)) return;    \
    const ShotDev& S = shots[s];                                                      \
    if (n >= S.nt) return; /* uniform over the workgroup */                           \
    const int NR = S.NR, NZ = S.NZ, nr = S.nr, pz = S.pz;                             \
    const Grid g{NR, NZ};                                                             \
    const long long cells = (long long)NR * NZ;                                       \
    const float dt = S.dt, idr = S.inv_dr, idz = S.inv_dz, dr = S.dr;                 \
    const float* __restrict__ prt = pml_r + S.pml_r_off;                              \
    const float* __restrict__ pzt = pml_z + S.pml_z_off

__device__ inline bool owned(int i, int k, int i0, int k0, int NR, int NZ)
{
    return i >= i0 && i < i0 + TI && k >= k0 && k < k0 + TK && i < NR && k < NZ;
}

// Each thread handles its owned cell in every region and at most one halo
// cell: NHD of the D-region (the four rows above and below the tile, then
// four columns on each side), NHP of the P-region (two of each).  The owned
// cells come first so that their values stay in the registers of the thread
// that finishes them.
constexpr int NHD = DN - TK * TI, NHP = PN - TK * TI;
static_assert(NHD <= TK * TI && NHP <= TK * TI, "one halo cell per thread");

__device__ inline int d_halo(int h)
{
    constexpr int band = 4 * DW;
    if (h < band) return h;
    if (h < 2 * band) return (TI + 4) * DW + (h - band);
    const int s = h - 2 * band, r = s >> 3, c = s & 7;
    return (4 + r) * DW + (c < 4 ? c : TK + c);
}

__device__ inline int p_halo(int h)
{
    constexpr int band = 2 * PW;
    if (h < band) return h;
    if (h < 2 * band) return (TI + 2) * PW + (h - band);
    const int s = h - 2 * band, r = s >> 2, c = s & 3;
    return (2 + r) * PW + (c < 2 ? c : TK + c);
}

// The stresses at (i, k) with the mirror rules, in the order of the forward's
// LDS planes: tau_rr, tau_tt (even), tau_rz (odd), tau_zz (even).
__device__ inline void tau4(const Grid& g, const float* __restrict__ F, long long cells, int i,
                            int k, float* t)
{
    t[0] = g.even(F + 2 * cells, i, k);
    t[1] = g.even(F + 3 * cells, i, k);
    t[2] = g.odd(F + 5 * cells, i, k);
    t[3] = g.even(F + 4 * cells, i, k);
}

// What a velocity update at (i, k) reads from memory besides the stresses:
// v^{n-1/2} and the buoyancies at the R and Z nodes (zero off the grid, and
// the R terms on the axis).
struct VelIn {
    float vr, vz, bR, bZ;
};

__device__ inline VelIn vel_in(const ShotDev& S, const float* __restrict__ F,
                               const float* __restrict__ rho, long long cells, int i, int k)
{
    VelIn V{0.f, 0.f, 0.f, 0.f};
    const int NR = S.NR, NZ = S.NZ;
    if (i >= 0 && i < NR && k >= 0 && k < NZ) {
        const long long c = (long long)i * NZ + k;
        const long long m = S.model_off + (long long)i * S.model_ld + k;
        const int k1 = k + 1 < NZ ? k + 1 : NZ - 1;
        V.vz = F[cells + c];
        V.bZ = 2.0f / (rho[m] + rho[m - k + k1]);
        if (i >= 1) {
            V.vr = F[c];
            V.bR = 2.0f / (rho[m - S.model_ld] + rho[m]);
        }
    }
    return V;
}

// ---------------------------------------------------------------------------
// Forward step.  State block as in the second-order kernels: 6 fields, then 4
// radial PML strips [A, C, E, H] of pr*NZ, then 4 axial strips [B, D, F, G]
// of NR*2pz.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(TK * TI)
k_fwd4(const ShotDev* __restrict__ shots, const int* __restrict__ tile_start, int nshot, int n,
       const float* __restrict__ lam, const float* __restrict__ mu,
       const float* __restrict__ rho, const float* __restrict__ wavelet,
       const int* __restrict__ rec_k, const float* __restrict__ pml_r,
       const float* __restrict__ pml_z, const float* __restrict__ sin,
       float* __restrict__ sout, float* __restrict__ traces, float* __restrict__ hist,
       long long cells_total)
{
    __shared__ float Ls[4][DN];  // tau_rr, tau_tt, tau_rz, tau_zz on the D-region
    __shared__ float Lv[2][PN];  // the new v_r, v_z on the P-region
    O4_PROLOGUE;
    const float* __restrict__ Fi = sin + S.fst_off;
    float* __restrict__ Fo = sout + S.fst_off;
    const long long LR = S.psir_len, LZ = S.psiz_len, oPR = 6 * cells, oPZ = oPR + 4 * LR;
    const int tid = (int)threadIdx.x;
    // this thread's owned cell, and its halo cell of each region (if any)
    const int i = i0 + (tid >> 6), k = k0 + (tid & 63);
    const bool ocell = i < NR && k < NZ;
    const bool hd = tid < NHD, hp = tid < NHP;
    const int ed = d_halo(hd ? tid : 0), ep = p_halo(hp ? tid : 0);
    const int di = i0 - 4 + ed / DW, dk = k0 - 4 + ed % DW;
    const int pi = i0 - 2 + ep / PW, pk = k0 - 2 + ep % PW;

    // ---- every load that does not depend on this step's LDS stages, issued
    // up front: the stresses of the D-region cells, v^{n-1/2} and the
    // buoyancies of the P-region cells, the moduli of the owned cell
    float td[2][4] = {};
    tau4(g, Fi, cells, i, k, td[0]);
    if (hd) tau4(g, Fi, cells, di, dk, td[1]);
    const VelIn V0 = vel_in(S, Fi, rho, cells, i, k);
    const VelIn V1 = hp ? vel_in(S, Fi, rho, cells, pi, pk) : VelIn{0.f, 0.f, 0.f, 0.f};
    const long long m = S.model_off + (long long)i * S.model_ld + k;
    const int k1 = k + 1 < NZ ? k + 1 : NZ - 1;
    float l = 0.f, u = 0.f, muS = 0.f;
    if (ocell) {
        l = lam[m];
        u = mu[m];
        if (i >= 1) {
            const long long mm = m - S.model_ld;
            muS = harm4(mu[mm], u, mu[mm - k + k1], mu[m - k + k1]);
        }
    }
    {
        const int e0 = ((tid >> 6) + 4) * DW + (tid & 63) + 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            Ls[q][e0] = td[0][q];
            if (hd) Ls[q][ed] = td[1][q];
        }
    }
    __syncthreads();
    const View trr{Ls[0], i0 - 4, k0 - 4, DW}, ttt{Ls[1], i0 - 4, k0 - 4, DW},
        trz{Ls[2], i0 - 4, k0 - 4, DW}, tzz{Ls[3], i0 - 4, k0 - 4, DW};

    // ---- velocities on the P-region (rows >= 0 inside the grid): the owned
    // cell, then the halo cell; only the owned one is stored
    auto velocity = [&](int i, int k, const VelIn& V, bool own, float& vrn, float& vzn) {
        vrn = vzn = 0.f;
        if (!(i >= 0 && i < NR && k >= 0 && k < NZ)) return;
        const long long c = (long long)i * NZ + k;
        const bool zp = k < pz || k >= NZ - pz;
        const int kk = zp ? (k < pz ? k : k - (NZ - 2 * pz)) : 0;
        if (i >= 1) {  // v_r at R(i, k)
            float Dr = (C1 * (trr(i, k) - trr(i - 1, k)) +
                        C2 * (trr(i + 1, k) - trr(i - 2, k))) * idr;
            float Dz = (C1 * (trz(i, k) - trz(i, k - 1)) +
                        C2 * (trz(i, k + 1) - trz(i, k - 2))) * idz;
            auto d = [&](int ii) { return trr(ii, k) - ttt(ii, k); };
            const float hoop = (G1 * (d(i) + d(i - 1)) + G2 * (d(i + 1) + d(i - 2))) / (i * dr);
            if (i >= nr) {  // A
                const long long q = oPR + (long long)(i - nr) * NZ + k;
                const float psi = prt[NR + i] * Fi[q] + prt[i] * Dr;
                if (own) Fo[q] = psi;
                Dr += psi;
            }
            if (zp) {  // B
                const long long q = oPZ + (long long)i * (2 * pz) + kk;
                const float psi = pzt[NZ + k] * Fi[q] + pzt[k] * Dz;
                if (own) Fo[q] = psi;
                Dz += psi;
            }
            vrn = V.vr + dt * V.bR * (Dr + Dz + hoop);
        }
        {  // v_z at Z(i, k)
            float Dr = (C1 * (trz(i + 1, k) - trz(i, k)) +
                        C2 * (trz(i + 2, k) - trz(i - 1, k))) * idr;
            float Dz = (C1 * (tzz(i, k + 1) - tzz(i, k)) +
                        C2 * (tzz(i, k + 2) - tzz(i, k - 1))) * idz;
            const float hoop = (G1 * (trz(i + 1, k) + trz(i, k)) +
                                G2 * (trz(i + 2, k) + trz(i - 1, k))) / ((i + 0.5f) * dr);
            if (i >= nr) {  // C
                const long long q = oPR + LR + (long long)(i - nr) * NZ + k;
                const float psi = prt[3 * NR + i] * Fi[q] + prt[2 * NR + i] * Dr;
                if (own) Fo[q] = psi;
                Dr += psi;
            }
            if (zp) {  // D
                const long long q = oPZ + LZ + (long long)i * (2 * pz) + kk;
                const float psi = pzt[3 * NZ + k] * Fi[q] + pzt[2 * NZ + k] * Dz;
                if (own) Fo[q] = psi;
                Dz += psi;
            }
            vzn = V.vz + dt * V.bZ * (Dr + Dz + hoop);
        }
        if (own) {
            if (i >= 1) Fo[c] = vrn;
            Fo[cells + c] = vzn;
            if (hist) {
                hist[S.cell_off + c] = vrn;
                hist[cells_total + S.cell_off + c] = vzn;
            }
        }
    };
    {
        float a, b;
        velocity(i, k, V0, ocell, a, b);
        const int e0 = ((tid >> 6) + 2) * PW + (tid & 63) + 2;
        Lv[0][e0] = a;
        Lv[1][e0] = b;
        if (hp) {
            velocity(pi, pk, V1, false, a, b);
            Lv[0][ep] = a;
            Lv[1][ep] = b;
        }
    }
    __syncthreads();
    // the mirror rows below the axis: v_r odd, v_z even (uniform: i0 is the
    // workgroup's)
    if (i0 == 0) {
        for (int e = tid; e < 2 * PW; e += TK * TI) {
            const int r = e / PW, q = e % PW;  // P-region row r is grid row r - 2
            const int im = r - 2;
            Lv[0][r * PW + q] = -Lv[0][(-im + 2) * PW + q];
            Lv[1][r * PW + q] = Lv[1][(-1 - im + 2) * PW + q];
        }
        __syncthreads();
    }
    if (!ocell) return;
    const View vr{Lv[0], i0 - 2, k0 - 2, PW}, vz{Lv[1], i0 - 2, k0 - 2, PW};
    const long long c = (long long)i * NZ + k;
    const bool zp = k < pz || k >= NZ - pz;
    const int kk = zp ? (k < pz ? k : k - (NZ - 2 * pz)) : 0;

    // ---- normal stresses at C(i, k)
    float err = (C1 * (vr(i + 1, k) - vr(i, k)) + C2 * (vr(i + 2, k) - vr(i - 1, k))) * idr;
    const float ett = (G1 * (vr(i + 1, k) + vr(i, k)) + G2 * (vr(i + 2, k) + vr(i - 1, k))) /
                      ((i + 0.5f) * dr);
    float ezz = (C1 * (vz(i, k) - vz(i, k - 1)) + C2 * (vz(i, k + 1) - vz(i, k - 2))) * idz;
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
    const float tr = err + ett + ezz;
    float nrr = trr(i, k) + dt * (l * tr + 2.0f * u * err);
    float ntt = ttt(i, k) + dt * (l * tr + 2.0f * u * ett);
    float nzz = tzz(i, k) + dt * (l * tr + 2.0f * u * ezz);
    if (i == 0 && k == S.src_k) {
        const float sv = AXIS_SRC * S.src_scale * wavelet[S.wave_off + n];
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
        float ez = (C1 * (vr(i, k + 1) - vr(i, k)) + C2 * (vr(i, k + 2) - vr(i, k - 1))) * idz;
        float er = (C1 * (vz(i, k) - vz(i - 1, k)) + C2 * (vz(i + 1, k) - vz(i - 2, k))) * idr;
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
        Fo[5 * cells + c] = trz(i, k) + dt * muS * (ez + er);
    }
}

// ---------------------------------------------------------------------------
// Adjoint step.  Adjoint state block as in the second-order kernels: 6
// fields, 5 radial strips [A-bar, C-bar, PhiT_r, PhiR_r, PhiH], 5 axial strips
// [B-bar, D-bar, PhiT_z, PhiZ_z, PhiG].
// ---------------------------------------------------------------------------

// The residual-injected adjoint stresses of a cell, the new Phi recursions of
// its PML memories and the drivers of the transposed stress update
// (sigma = C a_tau plus the PML terms).
struct AdjPoint {
    float trr, ttt, tzz, trz, sa;
    float pTr, pRr, pTz, pZz, pG, pH;
    float a_rh, a_zi, a_zh, a_ri;
    float Err, Ett, Ezz, Ez, Er;
};

__device__ inline AdjPoint adj_point(const ShotDev& S, int i, int k, int n,
                                     const float* __restrict__ lam, const float* __restrict__ mu,
                                     const int* __restrict__ rec_k,
                                     const float* __restrict__ resid,
                                     const float* __restrict__ prt,
                                     const float* __restrict__ pzt, const float* __restrict__ Ai)
{
    const int NR = S.NR, NZ = S.NZ, nr = S.nr, pz = S.pz;
    const long long cells = (long long)NR * NZ, c = (long long)i * NZ + k;
    const long long LR = S.psir_len, LZ = S.psiz_len, oPR = 6 * cells, oPZ = oPR + 5 * LR;
    const bool zp = k < pz || k >= NZ - pz;
    const int kk = zp ? (k < pz ? k : k - (NZ - 2 * pz)) : 0;
    const float dt = S.dt;
    const long long m = S.model_off + (long long)i * S.model_ld + k;
    AdjPoint P;
    P.trr = Ai[2 * cells + c];
    P.ttt = Ai[3 * cells + c];
    P.tzz = Ai[4 * cells + c];
    if (i == 0) {
        float inj = 0.f;
        for (int j = 0; j < S.nrec; ++j)
            if (rec_k[S.rec_off + j] == k) inj += resid[S.trace_off + (long long)j * S.nt + n];
        inj *= (1.0f / 3.0f);
        P.trr += inj;
        P.ttt += inj;
        P.tzz += inj;
    }
    const float l = lam[m], u = mu[m];
    P.sa = P.trr + P.ttt + P.tzz;
    P.Err = dt * (l * P.sa + 2.0f * u * P.trr);
    P.Ett = dt * (l * P.sa + 2.0f * u * P.ttt);
    P.Ezz = dt * (l * P.sa + 2.0f * u * P.tzz);
    P.pTr = P.pRr = P.pTz = P.pZz = P.pG = P.pH = 0.f;
    P.a_rh = P.a_zh = P.a_ri = 0.f;
    P.a_zi = zp ? pzt[k] : 0.f;
    if (i >= nr) {
        const long long q = oPR + (long long)(i - nr) * NZ + k;
        const float b = prt[3 * NR + i];
        P.a_rh = prt[2 * NR + i];
        P.pTr = dt * P.sa + b * Ai[q + 2 * LR];
        P.pRr = dt * P.trr + b * Ai[q + 3 * LR];
        P.Err += P.a_rh * (l * P.pTr + 2.0f * u * P.pRr);
    }
    if (zp) {
        const long long q = oPZ + (long long)i * (2 * pz) + kk;
        const float b = pzt[NZ + k];
        P.pTz = dt * P.sa + b * Ai[q + 2 * LZ];
        P.pZz = dt * P.tzz + b * Ai[q + 3 * LZ];
        P.Ezz += P.a_zi * (l * P.pTz + 2.0f * u * P.pZz);
    }
    P.trz = P.Ez = P.Er = 0.f;
    if (i >= 1) {
        P.trz = Ai[5 * cells + c];
        const int k1 = k + 1 < NZ ? k + 1 : NZ - 1;
        const long long mm = m - S.model_ld;
        const float muS = harm4(mu[mm], u, mu[mm - k + k1], mu[m - k + k1]);
        P.Ez = P.Er = dt * muS * P.trz;
        if (zp) {
            const long long q = oPZ + 4 * LZ + (long long)i * (2 * pz) + kk;
            P.a_zh = pzt[2 * NZ + k];
            P.pG = dt * P.trz + pzt[3 * NZ + k] * Ai[q];
            P.Ez += P.a_zh * muS * P.pG;
        }
        if (i >= nr) {
            const long long q = oPR + 4 * LR + (long long)(i - nr) * NZ + k;
            P.a_ri = prt[i];
            P.pH = dt * P.trz + prt[NR + i] * Ai[q];
            P.Er += P.a_ri * muS * P.pH;
        }
    }
    return P;
}

// Transposed gathers from an LDS region of per-node values (zero outside the
// grid and at negative rows).  "lo": the forward stencil's output at integer
// row i read the inputs at rows i-1, i (and i-2, i+1 for C2); "hi": the output
// at half row i + 1/2 read rows i, i+1 (and i-1, i+2).  The transposes at
// input row j:
//   Dlo: C1 (P[j] - P[j+1]) + C2 (P[j-1] - P[j+2]),  Ilo: same with +,
//   Dhi: C1 (P[j-1] - P[j]) + C2 (P[j-2] - P[j+1]),  Ihi: same with +.
// The folded radial forms add the gather at the mirrored logical row: an even
// (half-position) input row j in {0, 1} receives row -1 - j, an odd
// (integer) input row 1 the negated gather of row -1.
struct Gather {
    __device__ static float Dlo_r(const View& T, int j, int k)
    {
        return C1 * (T.at(j, k) - T.at(j + 1, k)) + C2 * (T.at(j - 1, k) - T.at(j + 2, k));
    }
    __device__ static float Ilo_r(const View& T, int j, int k)
    {
        return G1 * (T.at(j, k) + T.at(j + 1, k)) + G2 * (T.at(j - 1, k) + T.at(j + 2, k));
    }
    __device__ static float Dhi_r(const View& T, int j, int k)
    {
        return C1 * (T.at(j - 1, k) - T.at(j, k)) + C2 * (T.at(j - 2, k) - T.at(j + 1, k));
    }
    __device__ static float Ihi_r(const View& T, int j, int k)
    {
        return G1 * (T.at(j - 1, k) + T.at(j, k)) + G2 * (T.at(j - 2, k) + T.at(j + 1, k));
    }
    __device__ static float Dlo_z(const View& T, int i, int j)
    {
        return C1 * (T(i, j) - T(i, j + 1)) + C2 * (T(i, j - 1) - T(i, j + 2));
    }
    __device__ static float Dhi_z(const View& T, int i, int j)
    {
        return C1 * (T(i, j - 1) - T(i, j)) + C2 * (T(i, j - 2) - T(i, j + 1));
    }
    __device__ static float Dlo_r_even(const View& T, int j, int k)
    {
        return Dlo_r(T, j, k) + (j <= 1 ? Dlo_r(T, -1 - j, k) : 0.f);
    }
    __device__ static float Ilo_r_even(const View& T, int j, int k)
    {
        return Ilo_r(T, j, k) + (j <= 1 ? Ilo_r(T, -1 - j, k) : 0.f);
    }
    __device__ static float Dhi_r_odd(const View& T, int j, int k)
    {
        return Dhi_r(T, j, k) - (j == 1 ? Dhi_r(T, -1, k) : 0.f);
    }
    __device__ static float Ihi_r_odd(const View& T, int j, int k)
    {
        return Ihi_r(T, j, k) - (j == 1 ? Ihi_r(T, -1, k) : 0.f);
    }
};

enum { D_ERR = 0, D_ETT, D_EZZ, D_EZ, D_ER, ND };
enum { P_UR = 0, P_HR, P_DZR, P_ZR, P_ZH, P_DZZ, NP };

// What the transposed velocity update at (i, k) reads from memory besides the
// drivers: the adjoint velocities and dt times the buoyancies at the R and Z
// nodes (zero off the grid, and the R terms on the axis).
struct AdjVelIn {
    float ar, az, fR, fZ;
};

__device__ inline AdjVelIn adj_vel_in(const ShotDev& S, const float* __restrict__ A,
                                      const float* __restrict__ rho, long long cells, int i, int k)
{
    AdjVelIn V{0.f, 0.f, 0.f, 0.f};
    const int NR = S.NR, NZ = S.NZ;
    const float dt = S.dt;
    if (i >= 0 && i < NR && k >= 0 && k < NZ) {
        const long long c = (long long)i * NZ + k;
        const long long m = S.model_off + (long long)i * S.model_ld + k;
        const int k1 = k + 1 < NZ ? k + 1 : NZ - 1;
        V.az = A[cells + c];
        V.fZ = dt * 2.0f / (rho[m] + rho[m - k + k1]);
        if (i >= 1) {
            V.ar = A[c];
            V.fR = dt * 2.0f / (rho[m - S.model_ld] + rho[m]);
        }
    }
    return V;
}

// X selects extra outputs as in the second-order adjoint: bit 0 the density
// correlation (the increment of the adjoint velocity from the transposed
// stress update times the stored v^{n+1/2}, at the R and Z nodes, into
// acc_rho), bit 1 the virtual-source pseudo-Hessian diagonal (the plain
// fourth-order strain rates of v^{n+1/2}, into acc_h).
template <int X>
__global__ void __launch_bounds__(TK * TI)
k_adj4(const ShotDev* __restrict__ shots, const int* __restrict__ tile_start, int nshot, int n,
       const float* __restrict__ lam, const float* __restrict__ mu,
       const float* __restrict__ rho, const int* __restrict__ rec_k,
       const float* __restrict__ resid, const float* __restrict__ pml_r,
       const float* __restrict__ pml_z, const float* __restrict__ ain,
       float* __restrict__ aout, const float* __restrict__ hist, float* __restrict__ acc,
       float* __restrict__ acc_rho, float* __restrict__ acc_h, long long cells_total)
{
    constexpr bool RHO = (X & 1) != 0, HES = (X & 2) != 0;
    __shared__ float Ld[ND][DN];  // drivers on the D-region
    __shared__ float Lp[NP][PN];  // products on the P-region
    __shared__ float Lh[2][PN];   // stored v_r, v_z on the P-region
    O4_PROLOGUE;
    const float* __restrict__ Ai = ain + S.ast_off;
    float* __restrict__ Ao = aout + S.ast_off;
    const long long LR = S.psir_len, LZ = S.psiz_len, oPR = 6 * cells, oPZ = oPR + 5 * LR;
    const int tid = (int)threadIdx.x;
    // this thread's owned cell, and its halo cell of each region (if any)
    const int i = i0 + (tid >> 6), k = k0 + (tid & 63);
    const bool ocell = i < NR && k < NZ;
    const bool hd = tid < NHD, hp = tid < NHP;
    const int ed = d_halo(hd ? tid : 0), ep = p_halo(hp ? tid : 0);
    const int di = i0 - 4 + ed / DW, dk = k0 - 4 + ed % DW;
    const int pi = i0 - 2 + ep / PW, pk = k0 - 2 + ep % PW;
    const int e0d = ((tid >> 6) + 4) * DW + (tid & 63) + 4;
    const int e0p = ((tid >> 6) + 2) * PW + (tid & 63) + 2;

    // ---- every load that does not depend on this step's LDS stages, issued
    // up front.  The owned cell's adjoint point is kept to the end; of the
    // halo cell only its drivers are needed.
    AdjPoint P{};
    if (ocell) P = adj_point(S, i, k, n, lam, mu, rec_k, resid, prt, pzt, Ai);
    float dh[ND] = {};
    if (hd && di >= 0 && di < NR && dk >= 0 && dk < NZ) {
        const AdjPoint Q = adj_point(S, di, dk, n, lam, mu, rec_k, resid, prt, pzt, Ai);
        dh[D_ERR] = Q.Err;
        dh[D_ETT] = Q.Ett;
        dh[D_EZZ] = Q.Ezz;
        dh[D_EZ] = Q.Ez;
        dh[D_ER] = Q.Er;
    }
    // the stored v^{n+1/2} on the P-region: v_r odd, v_z even across the axis
    const float* __restrict__ hr = hist + S.cell_off;
    const float* __restrict__ hz = hist + cells_total + S.cell_off;
    const float h0r = g.odd(hr, i, k), h0z = g.even(hz, i, k);
    float h1r = 0.f, h1z = 0.f;
    if (hp) {
        h1r = g.odd(hr, pi, pk);
        h1z = g.even(hz, pi, pk);
    }
    const AdjVelIn V0 = adj_vel_in(S, Ai, rho, cells, i, k);
    const AdjVelIn V1 = hp ? adj_vel_in(S, Ai, rho, cells, pi, pk) : AdjVelIn{0.f, 0.f, 0.f, 0.f};
    const long long c = (long long)i * NZ + k;
    float* ga = acc + S.cell_off + c;
    float g0 = 0.f, g1 = 0.f, g2 = 0.f, g3 = 0.f, gR = 0.f, gZ = 0.f, hL = 0.f, hM = 0.f;
    float* gr = RHO ? acc_rho + S.cell_off + c : nullptr;
    float* gh = HES ? acc_h + S.cell_off + c : nullptr;
    if (ocell) {
        g0 = ga[0];
        g1 = ga[cells_total];
        g3 = ga[3 * cells_total];
        if (i >= 1) g2 = ga[2 * cells_total];
        if constexpr (RHO) {
            if (i >= 1) gR = gr[0];
            gZ = gr[cells_total];
        }
        if constexpr (HES) {
            hL = gh[0];
            hM = gh[cells_total];
        }
    }
    Ld[D_ERR][e0d] = P.Err;
    Ld[D_ETT][e0d] = P.Ett;
    Ld[D_EZZ][e0d] = P.Ezz;
    Ld[D_EZ][e0d] = P.Ez;
    Ld[D_ER][e0d] = P.Er;
    Lh[0][e0p] = h0r;
    Lh[1][e0p] = h0z;
    if (hd) {
#pragma unroll
        for (int q = 0; q < ND; ++q) Ld[q][ed] = dh[q];
    }
    if (hp) {
        Lh[0][ep] = h1r;
        Lh[1][ep] = h1z;
    }
    __syncthreads();
    const View Err{Ld[D_ERR], i0 - 4, k0 - 4, DW}, Ett{Ld[D_ETT], i0 - 4, k0 - 4, DW},
        Ezz{Ld[D_EZZ], i0 - 4, k0 - 4, DW}, Ez{Ld[D_EZ], i0 - 4, k0 - 4, DW},
        Er{Ld[D_ER], i0 - 4, k0 - 4, DW};

    // ---- adjoint velocities and the products of the transposed velocity
    // update on the P-region: the owned cell (stored), then the halo cell
    float dar = 0.f, daz = 0.f;  // the owned cell's a_v increments (density)
    auto products = [&](int i, int k, const AdjVelIn& V, bool own, float* p) {
#pragma unroll
        for (int q = 0; q < NP; ++q) p[q] = 0.f;
        if (!(i >= 0 && i < NR && k >= 0 && k < NZ)) return;
        const long long c = (long long)i * NZ + k;
        const bool zp = k < pz || k >= NZ - pz;
        const int kk = zp ? (k < pz ? k : k - (NZ - 2 * pz)) : 0;
        // a_v_r at R(i, k), i >= 1: the stress update read v_r through e_rr
        // (C, half output), e_tt (C, I / r) and e_z (S, axial half output)
        if (i >= 1) {
            auto q = [&](int ii) { return Ett.at(ii, k) * (1.0f / ((ii + 0.5f) * dr)); };
            float it = G1 * (q(i - 1) + q(i)) + G2 * (q(i - 2) + q(i + 1));
            if (i == 1) it -= G2 * q(0);  // mirror of row -1
            const float avr = V.ar + Gather::Dhi_r_odd(Err, i, k) * idr + it +
                              Gather::Dhi_z(Ez, i, k) * idz;
            if (own) Ao[c] = avr;
            if (RHO && own)
                dar = Gather::Dhi_r_odd(Err, i, k) * idr + it + Gather::Dhi_z(Ez, i, k) * idz;
            const float W1 = V.fR * avr;
            float aDr = W1, aDz = W1;
            if (i >= nr) {  // A-bar
                const long long qq = oPR + (long long)(i - nr) * NZ + k;
                const float v = Ai[qq] + W1;
                if (own) Ao[qq] = prt[NR + i] * v;
                aDr += prt[i] * v;
            }
            if (zp) {  // B-bar
                const long long qq = oPZ + (long long)i * (2 * pz) + kk;
                const float v = Ai[qq] + W1;
                if (own) Ao[qq] = pzt[NZ + k] * v;
                aDz += pzt[k] * v;
            }
            p[P_UR] = aDr;
            p[P_HR] = W1 / (i * dr);
            p[P_DZR] = aDz;
        }
        // a_v_z at Z(i, k): read through e_zz (C, axial integer output)
        // and e_r (S, radial integer output)
        const float avz = V.az + Gather::Dlo_z(Ezz, i, k) * idz +
                          Gather::Dlo_r_even(Er, i, k) * idr;
        if (own) Ao[cells + c] = avz;
        if (RHO && own) daz = Gather::Dlo_z(Ezz, i, k) * idz + Gather::Dlo_r_even(Er, i, k) * idr;
        const float W2 = V.fZ * avz;
        float aDr = W2, aDz = W2;
        if (i >= nr) {  // C-bar
            const long long qq = oPR + LR + (long long)(i - nr) * NZ + k;
            const float v = Ai[qq] + W2;
            if (own) Ao[qq] = prt[3 * NR + i] * v;
            aDr += prt[2 * NR + i] * v;
        }
        if (zp) {  // D-bar
            const long long qq = oPZ + LZ + (long long)i * (2 * pz) + kk;
            const float v = Ai[qq] + W2;
            if (own) Ao[qq] = pzt[3 * NZ + k] * v;
            aDz += pzt[2 * NZ + k] * v;
        }
        p[P_ZR] = aDr;
        p[P_ZH] = W2 / ((i + 0.5f) * dr);
        p[P_DZZ] = aDz;
    };
    {
        float p[NP];
        products(i, k, V0, ocell, p);
#pragma unroll
        for (int q = 0; q < NP; ++q) Lp[q][e0p] = p[q];
        if (hp) {
            products(pi, pk, V1, false, p);
#pragma unroll
            for (int q = 0; q < NP; ++q) Lp[q][ep] = p[q];
        }
    }
    __syncthreads();

    // ---- the owned cell: adjoint stresses, PML memories, Eq. 7-8
    if (!ocell) return;
    const bool zp = k < pz || k >= NZ - pz;
    const int kk = zp ? (k < pz ? k : k - (NZ - 2 * pz)) : 0;
    if (i >= nr) {
        const long long q = oPR + (long long)(i - nr) * NZ + k;
        Ao[q + 2 * LR] = P.pTr;
        Ao[q + 3 * LR] = P.pRr;
        if (i >= 1) Ao[oPR + 4 * LR + (long long)(i - nr) * NZ + k] = P.pH;
    }
    if (zp) {
        const long long q = oPZ + (long long)i * (2 * pz) + kk;
        Ao[q + 2 * LZ] = P.pTz;
        Ao[q + 3 * LZ] = P.pZz;
        if (i >= 1) Ao[q + 4 * LZ] = P.pG;
    }
    const View UR{Lp[P_UR], i0 - 2, k0 - 2, PW}, HR{Lp[P_HR], i0 - 2, k0 - 2, PW},
        DZR{Lp[P_DZR], i0 - 2, k0 - 2, PW}, ZR{Lp[P_ZR], i0 - 2, k0 - 2, PW},
        ZH{Lp[P_ZH], i0 - 2, k0 - 2, PW}, DZZ{Lp[P_DZZ], i0 - 2, k0 - 2, PW};
    // C node: the velocity update read tau_rr (D and I at R nodes, integer
    // outputs from half inputs), tau_tt (-I at R nodes), tau_zz (Z nodes, axial
    // half outputs)
    const float h = Gather::Ilo_r_even(HR, i, k);
    Ao[2 * cells + c] = P.trr + Gather::Dlo_r_even(UR, i, k) * idr + h;
    Ao[3 * cells + c] = P.ttt - h;
    Ao[4 * cells + c] = P.tzz + Gather::Dhi_z(DZZ, i, k) * idz;
    // S node: tau_rz read by v_r (axial integer output from half inputs) and by
    // v_z (radial half outputs from integer inputs, D and I)
    Ao[5 * cells + c] = i >= 1 ? P.trz + Gather::Dlo_z(DZR, i, k) * idz +
                                     Gather::Dhi_r_odd(ZR, i, k) * idr +
                                     Gather::Ihi_r_odd(ZH, i, k)
                               : 0.f;

    // Eq. 7-8 with the strain rates of the stored v^{n+1/2}
    const View vrh{Lh[0], i0 - 2, k0 - 2, PW}, vzh{Lh[1], i0 - 2, k0 - 2, PW};
    const float vr0 = vrh(i, k), vr1 = vrh(i + 1, k);
    const float err = (C1 * (vr1 - vr0) + C2 * (vrh(i + 2, k) - vrh(i - 1, k))) * idr;
    const float ett = (G1 * (vr1 + vr0) + G2 * (vrh(i + 2, k) + vrh(i - 1, k))) / ((i + 0.5f) * dr);
    const float vz0 = vzh(i, k), vzm = vzh(i, k - 1);
    const float ezz = (C1 * (vz0 - vzm) + C2 * (vzh(i, k + 1) - vzh(i, k - 2))) * idz;
    const float dgl = dt * (err + ett + ezz) * P.sa + P.a_rh * err * P.pTr + P.a_zi * ezz * P.pTz;
    const float dgm = 2.0f * dt * (err * P.trr + ett * P.ttt + ezz * P.tzz) +
                      2.0f * (P.a_rh * err * P.pRr + P.a_zi * ezz * P.pZz);
    const float ur = 0.5f * (vr0 + vr1), uz = 0.5f * (vzm + vz0);
    ga[0] = g0 + dgl;
    ga[cells_total] = g1 + dgm;
    ga[3 * cells_total] = g3 + dt * (ur * ur + uz * uz);
    float es = 0.f;
    if (i >= 1) {
        const float ez = (C1 * (vrh(i, k + 1) - vr0) + C2 * (vrh(i, k + 2) - vrh(i, k - 1))) * idz;
        const float er = (C1 * (vz0 - vzh(i - 1, k)) + C2 * (vzh(i + 1, k) - vzh(i - 2, k))) * idr;
        ga[2 * cells_total] = g2 + (dt * (ez + er) * P.trz + P.a_zh * ez * P.pG + P.a_ri * er * P.pH);
        es = ez + er;
    }
    (void)es;
    if constexpr (RHO) {
        if (i >= 1) gr[0] = gR + dar * vr0;
        gr[cells_total] = gZ + daz * vz0;
    }
    if constexpr (HES) {
        const float dv = err + ett + ezz;
        gh[0] = hL + dt * dt * (3.0f * dv * dv);
        gh[cells_total] = hM + dt * dt * (4.0f * (err * err + ett * ett + ezz * ezz) + es * es);
    }
}

#undef O4_PROLOGUE

}  // namespace o4
}  // namespace bhfwi
