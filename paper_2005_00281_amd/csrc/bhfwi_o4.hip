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
// Each kernel works on tiles of TK = 64 axial by TI = 8 radial cells, one
// thread per cell in a 512-thread workgroup: the input planes a tile reads
// with its neighbours are staged in LDS once, with a two-cell halo and the
// boundary rules applied while staging, and every stencil then reads LDS.
// The forward step is two kernels (velocities, then stresses).  The adjoint is three, the
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

constexpr int TK = 64, TI = 8, HW = TK + 4, HH = TI + 4, HN = HW * HH;

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
    // a per-node product (zero outside the grid, no mirror: the fold does it)
    __device__ float at(const float* __restrict__ p, int i, int k) const
    {
        if (k < 0 || k >= NZ || i < 0 || i >= NR) return 0.f;
        return p[(long long)i * NZ + k];
    }
};

enum { EVEN = 0, ODD, AT };

// Stage one plane of the tile (rows i0-2 .. i0+TI+1, columns k0-2 ..
// k0+TK+1) in LDS with the boundary rule of its kind.
template <int MODE>
__device__ inline void stage(float* __restrict__ L, const Grid& g, const float* __restrict__ p,
                             int i0, int k0)
{
    for (int e = threadIdx.x; e < HN; e += blockDim.x) {
        const int i = i0 - 2 + e / HW, k = k0 - 2 + e % HW;
        L[e] = MODE == EVEN ? g.even(p, i, k) : MODE == ODD ? g.odd(p, i, k) : g.at(p, i, k);
    }
}

// A staged plane read at grid cell (i, k), |i - i0 - TI/2| and |k - k0 - TK/2|
// within the halo; products (no mirror) read zero at negative rows.
struct Tile {
    const float* L;
    int i0, k0;
    __device__ float operator()(int i, int k) const
    {
        return L[(i - i0 + 2) * HW + (k - k0 + 2)];
    }
    __device__ float at(int i, int k) const { return i < 0 ? 0.f : (*this)(i, k); }
};

__device__ inline float harm4(float a, float b, float c, float d)
{
    return (a > 0.f && b > 0.f && c > 0.f && d > 0.f)
               ? 4.0f / (1.0f / a + 1.0f / b + 1.0f / c + 1.0f / d)
               : 0.0f;
}

// The tile prologue shared by the kernels: shot, tile origin and this
// thread's cell; threads past the grid still take part in the staging.
#define O4_PROLOGUE                                                                   \
    int s, i0, k0;                                                                    \
    if (!tile_of(shots, tile_start, nshot, (int)blockIdx.x, &s, &i0, &k0)) return;    \
    const ShotDev& S = shots[s];                                                      \
    if (n >= S.nt) return; /* uniform over the workgroup */                           \
    const int i = i0 + (int)(threadIdx.x >> 6), k = k0 + (int)(threadIdx.x & 63);     \
    const int NR = S.NR, NZ = S.NZ, nr = S.nr, pz = S.pz;                             \
    const bool own = i < NR && k < NZ;                                                \
    const Grid g{NR, NZ};                                                             \
    const long long cells = (long long)NR * NZ, c = (long long)i * NZ + k;            \
    const bool zp = k < pz || k >= NZ - pz;                                           \
    const int kk = zp ? (k < pz ? k : k - (NZ - 2 * pz)) : 0;                         \
    const float dt = S.dt, idr = S.inv_dr, idz = S.inv_dz, dr = S.dr;                 \
    const long long m = S.model_off + (long long)i * S.model_ld + k;                  \
    const float* __restrict__ prt = pml_r + S.pml_r_off;                              \
    const float* __restrict__ pzt = pml_z + S.pml_z_off

// ---------------------------------------------------------------------------
// Forward.  State block as in the second-order kernels: 6 fields, then 4
// radial PML strips [A, C, E, H] of pr*NZ, then 4 axial strips [B, D, F, G]
// of NR*2pz.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(512)
k_fwd4_vel(const ShotDev* __restrict__ shots, const int* __restrict__ tile_start, int nshot,
           int n, const float* __restrict__ rho, const float* __restrict__ pml_r,
           const float* __restrict__ pml_z, const float* __restrict__ sin,
           float* __restrict__ sout, float* __restrict__ hist, long long cells_total)
{
    __shared__ float L[4][HN];
    O4_PROLOGUE;
    const float* __restrict__ Fi = sin + S.fst_off;
    float* __restrict__ Fo = sout + S.fst_off;
    stage<EVEN>(L[0], g, Fi + 2 * cells, i0, k0);
    stage<EVEN>(L[1], g, Fi + 3 * cells, i0, k0);
    stage<ODD>(L[2], g, Fi + 5 * cells, i0, k0);
    stage<EVEN>(L[3], g, Fi + 4 * cells, i0, k0);
    __syncthreads();
    if (!own) return;
    const Tile trr{L[0], i0, k0}, ttt{L[1], i0, k0}, trz{L[2], i0, k0}, tzz{L[3], i0, k0};
    const long long LR = S.psir_len, LZ = S.psiz_len, oPR = 6 * cells, oPZ = oPR + 4 * LR;

    // ---- v_r at R(i, k), i >= 1
    float vrn = 0.f;
    if (i >= 1) {
        float Dr = (C1 * (trr(i, k) - trr(i - 1, k)) + C2 * (trr(i + 1, k) - trr(i - 2, k))) * idr;
        float Dz = (C1 * (trz(i, k) - trz(i, k - 1)) + C2 * (trz(i, k + 1) - trz(i, k - 2))) * idz;
        auto d = [&](int ii) { return trr(ii, k) - ttt(ii, k); };
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
        vrn = Fi[c] + dt * bR * (Dr + Dz + hoop);
        Fo[c] = vrn;
    }
    // ---- v_z at Z(i, k)
    float Dr = (C1 * (trz(i + 1, k) - trz(i, k)) + C2 * (trz(i + 2, k) - trz(i - 1, k))) * idr;
    float Dz = (C1 * (tzz(i, k + 1) - tzz(i, k)) + C2 * (tzz(i, k + 2) - tzz(i, k - 1))) * idz;
    const float hoop = (G1 * (trz(i + 1, k) + trz(i, k)) + G2 * (trz(i + 2, k) + trz(i - 1, k))) /
                       ((i + 0.5f) * dr);
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
    const float vzn = Fi[cells + c] + dt * bZ * (Dr + Dz + hoop);
    Fo[cells + c] = vzn;
    if (hist) {
        hist[S.cell_off + c] = vrn;
        hist[cells_total + S.cell_off + c] = vzn;
    }
}

__global__ void __launch_bounds__(512)
k_fwd4_str(const ShotDev* __restrict__ shots, const int* __restrict__ tile_start, int nshot,
           int n, const float* __restrict__ lam, const float* __restrict__ mu,
           const float* __restrict__ wavelet, const int* __restrict__ rec_k,
           const float* __restrict__ pml_r, const float* __restrict__ pml_z,
           const float* __restrict__ sin, float* __restrict__ sout, float* __restrict__ traces)
{
    __shared__ float L[2][HN];
    O4_PROLOGUE;
    const float* __restrict__ Fi = sin + S.fst_off;
    float* __restrict__ Fo = sout + S.fst_off;
    stage<ODD>(L[0], g, Fo, i0, k0);           // the new v_r
    stage<EVEN>(L[1], g, Fo + cells, i0, k0);  // the new v_z
    __syncthreads();
    if (!own) return;
    const Tile vr{L[0], i0, k0}, vz{L[1], i0, k0};
    const long long LR = S.psir_len, LZ = S.psiz_len, oPR = 6 * cells, oPZ = oPR + 4 * LR;

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

__global__ void __launch_bounds__(512)
k_adj4_drivers(const ShotDev* __restrict__ shots, const int* __restrict__ tile_start, int nshot,
               int n, const float* __restrict__ lam, const float* __restrict__ mu,
               const int* __restrict__ rec_k, const float* __restrict__ resid,
               const float* __restrict__ pml_r, const float* __restrict__ pml_z,
               const float* __restrict__ ain, float* __restrict__ aout,
               const float* __restrict__ hist, float* __restrict__ scr,
               float* __restrict__ acc, long long cells_total)
{
    __shared__ float L[2][HN];
    O4_PROLOGUE;
    stage<ODD>(L[0], g, hist + S.cell_off, i0, k0);
    stage<EVEN>(L[1], g, hist + cells_total + S.cell_off, i0, k0);
    __syncthreads();
    if (!own) return;
    const Tile vrh{L[0], i0, k0}, vzh{L[1], i0, k0};
    const float* __restrict__ Ai = ain + S.ast_off;
    float* __restrict__ Ao = aout + S.ast_off;
    const long long LR = S.psir_len, LZ = S.psiz_len, oPR = 6 * cells, oPZ = oPR + 5 * LR;
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
    const float vr0 = vrh(i, k), vr1 = vrh(i + 1, k);
    const float err = (C1 * (vr1 - vr0) + C2 * (vrh(i + 2, k) - vrh(i - 1, k))) * idr;
    const float ett = (G1 * (vr1 + vr0) + G2 * (vrh(i + 2, k) + vrh(i - 1, k))) / ((i + 0.5f) * dr);
    const float vz0 = vzh(i, k), vzm = vzh(i, k - 1);
    const float ezz = (C1 * (vz0 - vzm) + C2 * (vzh(i, k + 1) - vzh(i, k - 2))) * idz;
    float dgl = dt * (err + ett + ezz) * sa + a_rh * err * pTr + a_zi * ezz * pTz;
    float dgm = 2.0f * dt * (err * trr + ett * ttt + ezz * tzz) +
                2.0f * (a_rh * err * pRr + a_zi * ezz * pZz);
    const float ur = 0.5f * (vr0 + vr1), uz = 0.5f * (vzm + vz0);
    float* ga = acc + S.cell_off + c;
    ga[0] += dgl;
    ga[cells_total] += dgm;
    ga[3 * cells_total] += dt * (ur * ur + uz * uz);
    if (i >= 1) {
        const float ez = (C1 * (vrh(i, k + 1) - vr0) + C2 * (vrh(i, k + 2) - vrh(i, k - 1))) * idz;
        const float er = (C1 * (vz0 - vzh(i - 1, k)) + C2 * (vzh(i + 1, k) - vzh(i - 2, k))) * idr;
        ga[2 * cells_total] += dt * (ez + er) * trz + a_zh * ez * pG + a_ri * er * pH;
    }
}

// Transposed gathers from a staged product plane T (zero outside the grid,
// no mirror).  "lo": the forward stencil's output at integer row i read the
// inputs at rows i-1, i (and i-2, i+1 for C2); "hi": the output at half row
// i + 1/2 read rows i, i+1 (and i-1, i+2).  The transposes at input row j:
//   Dlo: C1 (P[j] - P[j+1]) + C2 (P[j-1] - P[j+2]),  Ilo: same with +,
//   Dhi: C1 (P[j-1] - P[j]) + C2 (P[j-2] - P[j+1]),  Ihi: same with +.
// The folded radial forms add the gather at the mirrored logical row: an even
// (half-position) input row j in {0, 1} receives row -1 - j, an odd
// (integer) input row 1 the negated gather of row -1.
struct Gather {
    __device__ static float Dlo_r(const Tile& T, int j, int k)
    {
        return C1 * (T.at(j, k) - T.at(j + 1, k)) + C2 * (T.at(j - 1, k) - T.at(j + 2, k));
    }
    __device__ static float Ilo_r(const Tile& T, int j, int k)
    {
        return G1 * (T.at(j, k) + T.at(j + 1, k)) + G2 * (T.at(j - 1, k) + T.at(j + 2, k));
    }
    __device__ static float Dhi_r(const Tile& T, int j, int k)
    {
        return C1 * (T.at(j - 1, k) - T.at(j, k)) + C2 * (T.at(j - 2, k) - T.at(j + 1, k));
    }
    __device__ static float Ihi_r(const Tile& T, int j, int k)
    {
        return G1 * (T.at(j - 1, k) + T.at(j, k)) + G2 * (T.at(j - 2, k) + T.at(j + 1, k));
    }
    __device__ static float Dlo_z(const Tile& T, int i, int j)
    {
        return C1 * (T(i, j) - T(i, j + 1)) + C2 * (T(i, j - 1) - T(i, j + 2));
    }
    __device__ static float Dhi_z(const Tile& T, int i, int j)
    {
        return C1 * (T(i, j - 1) - T(i, j)) + C2 * (T(i, j - 2) - T(i, j + 1));
    }
    __device__ static float Dlo_r_even(const Tile& T, int j, int k)
    {
        return Dlo_r(T, j, k) + (j <= 1 ? Dlo_r(T, -1 - j, k) : 0.f);
    }
    __device__ static float Ilo_r_even(const Tile& T, int j, int k)
    {
        return Ilo_r(T, j, k) + (j <= 1 ? Ilo_r(T, -1 - j, k) : 0.f);
    }
    __device__ static float Dhi_r_odd(const Tile& T, int j, int k)
    {
        return Dhi_r(T, j, k) - (j == 1 ? Dhi_r(T, -1, k) : 0.f);
    }
    __device__ static float Ihi_r_odd(const Tile& T, int j, int k)
    {
        return Ihi_r(T, j, k) - (j == 1 ? Ihi_r(T, -1, k) : 0.f);
    }
};

__global__ void __launch_bounds__(512)
k_adj4_velocity(const ShotDev* __restrict__ shots, const int* __restrict__ tile_start,
                int nshot, int n, const float* __restrict__ rho,
                const float* __restrict__ pml_r, const float* __restrict__ pml_z,
                const float* __restrict__ ain, float* __restrict__ aout,
                float* __restrict__ scr, long long cells_total)
{
    __shared__ float L[5][HN];
    O4_PROLOGUE;
    float* __restrict__ base = scr + S.cell_off;
    stage<AT>(L[0], g, base + D_ERR * cells_total, i0, k0);
    stage<AT>(L[1], g, base + D_ETT * cells_total, i0, k0);
    stage<AT>(L[2], g, base + D_EZZ * cells_total, i0, k0);
    stage<AT>(L[3], g, base + D_EZ * cells_total, i0, k0);
    stage<AT>(L[4], g, base + D_ER * cells_total, i0, k0);
    __syncthreads();
    if (!own) return;
    const Tile Err{L[0], i0, k0}, Ett{L[1], i0, k0}, Ezz{L[2], i0, k0}, Ez{L[3], i0, k0},
        Er{L[4], i0, k0};
    const float* __restrict__ Ai = ain + S.ast_off;
    float* __restrict__ Ao = aout + S.ast_off;
    const long long LR = S.psir_len, LZ = S.psiz_len, oPR = 6 * cells, oPZ = oPR + 5 * LR;

    // ---- a_v_r at R(i, k), i >= 1: the stress update read v_r through e_rr
    // (C, half output), e_tt (C, I / r) and e_z (S, axial half output)
    float UR = 0.f, HR = 0.f, DZR = 0.f;
    if (i >= 1) {
        // e_tt carries 1/r_C: gather Ett / r_C
        auto q = [&](int ii) { return Ett.at(ii, k) * (1.0f / ((ii + 0.5f) * dr)); };
        float it = G1 * (q(i - 1) + q(i)) + G2 * (q(i - 2) + q(i + 1));
        if (i == 1) it -= G2 * q(0);  // mirror of row -1
        const float dar = Gather::Dhi_r_odd(Err, i, k) * idr + it + Gather::Dhi_z(Ez, i, k) * idz;
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
    const float daz = Gather::Dlo_z(Ezz, i, k) * idz + Gather::Dlo_r_even(Er, i, k) * idr;
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

__global__ void __launch_bounds__(512)
k_adj4_stress(const ShotDev* __restrict__ shots, const int* __restrict__ tile_start, int nshot,
              int n, const float* __restrict__ pml_r, const float* __restrict__ pml_z,
              float* __restrict__ aout, const float* __restrict__ scr, long long cells_total)
{
    __shared__ float L[6][HN];
    O4_PROLOGUE;
    const float* base = scr + S.cell_off;
    for (int q = 0; q < 6; ++q) stage<AT>(L[q], g, base + (P_UR + q) * cells_total, i0, k0);
    __syncthreads();
    if (!own) return;
    const Tile UR{L[0], i0, k0}, HR{L[1], i0, k0}, DZR{L[2], i0, k0}, ZR{L[3], i0, k0},
        ZH{L[4], i0, k0}, DZZ{L[5], i0, k0};
    float* __restrict__ Ao = aout + S.ast_off;
    (void)m; (void)prt; (void)pzt; (void)kk; (void)dt; (void)dr; (void)nr;
    // C node: the velocity update read tau_rr (D and I at R nodes, integer
    // outputs from half inputs), tau_tt (-I at R nodes), tau_zz (Z nodes, axial
    // half outputs)
    const float h = Gather::Ilo_r_even(HR, i, k);
    Ao[2 * cells + c] += Gather::Dlo_r_even(UR, i, k) * idr + h;
    Ao[3 * cells + c] -= h;
    Ao[4 * cells + c] += Gather::Dhi_z(DZZ, i, k) * idz;
    // S node: tau_rz read by v_r (axial integer output from half inputs) and by
    // v_z (radial half outputs from integer inputs, D and I)
    if (i >= 1)
        Ao[5 * cells + c] += Gather::Dlo_z(DZR, i, k) * idz + Gather::Dhi_r_odd(ZR, i, k) * idr +
                             Gather::Ihi_r_odd(ZH, i, k);
}

#undef O4_PROLOGUE

}  // namespace o4
}  // namespace bhfwi
