// bhfwi_semblance.hip -- starting-model construction: slowness-time coherence
// (semblance) of on-axis receiver gathers, coherence peak picking in a
// slowness band, and the radial interpolation of the picked velocities
// (Introduction; Numerical Examples section, Fig. 3-4).
//
// k_semblance: one workgroup per (gather, slowness, chunk of windows).  It
// first forms, for every sample of the chunk's time range, the squared stack
// of the moveout-corrected receivers and their energy (receiver m read
// p*offset_m/dt samples later, linearly interpolated, zero outside the
// record) into LDS, turns both series into prefix sums in double in place (a
// workgroup scan), and then takes every window's sums as a difference of two
// prefix values.  The time range of a chunk is at most kSemSpan samples, so
// the LDS footprint does not depend on the record length.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "bhfwi.h"

namespace bhfwi {

constexpr int kSemSpan = 2048;  // samples staged per workgroup
constexpr int kSemThreads = 256;
constexpr int kSemPer = kSemSpan / kSemThreads;  // samples per thread in the scan

__global__ void __launch_bounds__(kSemThreads)
k_semblance(int nrec, int nt, const float* __restrict__ traces, float dt,
            const float* __restrict__ offset, float p0, float dp, int ntau, int stride, int win,
            int chunk, float* __restrict__ coh, float* __restrict__ energy)
{
    // Ps[k], Pe[k]: first the squared stack and the energy of sample
    // n_lo + k - 1, then (in place) their prefix sums over samples < n_lo + k
    __shared__ double Ps[kSemSpan + 1];
    __shared__ double Pe[kSemSpan + 1];
    __shared__ double Ts[kSemThreads], Te[kSemThreads];  // per-thread totals, scanned
    __shared__ int Lq[64];                 // per receiver: whole samples of the shift
    __shared__ float Lf[64];               // and its fraction
    const int j = blockIdx.x, g = blockIdx.y;
    const int i0 = blockIdx.z * chunk;
    const int i1 = min(ntau, i0 + chunk);
    if (i0 >= i1) return;  // uniform
    const int np = gridDim.x;
    const float* __restrict__ x = traces + (long long)g * nrec * nt;
    if ((int)threadIdx.x < nrec) {
        // the shift p offset / dt in double, once per receiver, split into
        // whole samples and a fraction (large shifts keep their fraction)
        const double s = ((double)p0 + j * (double)dp) *
                         (double)offset[(long long)g * nrec + threadIdx.x] / (double)dt;
        const double fl = floor(s);
        Lq[threadIdx.x] = (int)fl;
        Lf[threadIdx.x] = (float)(s - fl);
    }
    __syncthreads();
    const int n_lo = i0 * stride;
    const int n_hi = min((i1 - 1) * stride + win, n_lo + kSemSpan);
    const int len = n_hi - n_lo;
    for (int n = n_lo + (int)threadIdx.x; n < n_hi; n += kSemThreads) {
        float st = 0.f, en = 0.f;
        for (int m = 0; m < nrec; ++m) {
            const int q = n + Lq[m];  // sample at or before the shifted time
            const float f = Lf[m];
            const float* __restrict__ xm = x + (long long)m * nt;
            const float a = (q >= 0 && q < nt) ? xm[q] : 0.f;
            const float b = (q + 1 >= 0 && q + 1 < nt) ? xm[q + 1] : 0.f;
            // the shifted time lies inside the record, or at its last sample
            float v = 0.f;
            if (q >= 0 && (q < nt - 1 || (q == nt - 1 && f == 0.f))) v = a + f * (b - a);
            st += v;
            en += v * v;
        }
        Ps[n - n_lo + 1] = (double)st * st;
        Pe[n - n_lo + 1] = en;
    }
    __syncthreads();
    // prefix sums in double: each thread totals kSemPer consecutive samples,
    // the totals are scanned (Hillis-Steele), then each thread turns its own
    // samples into running sums
    const int t0 = threadIdx.x * kSemPer + 1;
    double ts = 0.0, te = 0.0;
    for (int q = 0; q < kSemPer; ++q)
        if (t0 + q <= len) {
            ts += Ps[t0 + q];
            te += Pe[t0 + q];
        }
    Ts[threadIdx.x] = ts;
    Te[threadIdx.x] = te;
    __syncthreads();
    for (int o = 1; o < kSemThreads; o <<= 1) {
        const double as = threadIdx.x >= (unsigned)o ? Ts[threadIdx.x - o] : 0.0;
        const double ae = threadIdx.x >= (unsigned)o ? Te[threadIdx.x - o] : 0.0;
        __syncthreads();
        Ts[threadIdx.x] += as;
        Te[threadIdx.x] += ae;
        __syncthreads();
    }
    double rs = Ts[threadIdx.x] - ts, re = Te[threadIdx.x] - te;  // exclusive
    for (int q = 0; q < kSemPer; ++q)
        if (t0 + q <= len) {
            rs += Ps[t0 + q];
            re += Pe[t0 + q];
            Ps[t0 + q] = rs;
            Pe[t0 + q] = re;
        }
    if (threadIdx.x == 0) {
        Ps[0] = 0.0;
        Pe[0] = 0.0;
    }
    __syncthreads();
    for (int i = i0 + (int)threadIdx.x; i < i1; i += kSemThreads) {
        const int a0 = i * stride - n_lo;
        const double num = Ps[a0 + win] - Ps[a0], den = Pe[a0 + win] - Pe[a0];
        const long long o = ((long long)g * np + j) * ntau + i;
        coh[o] = den > 0.0 ? (float)(num / (nrec * den)) : 0.f;
        if (energy) energy[o] = (float)den;
    }
}

__global__ void k_sem_fill(float* __restrict__ p, int n, float v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Largest window energy of each gather, into emax[g] (non-negative floats
// order as their bit patterns); grid (slices, gathers).
__global__ void __launch_bounds__(kSemThreads)
k_sem_emax(long long cells, const float* __restrict__ energy, float* __restrict__ emax)
{
    __shared__ float S[kSemThreads];
    const int g = blockIdx.y;
    const float* __restrict__ e = energy + (long long)g * cells;
    float m = 0.f;
    for (long long q = (long long)blockIdx.x * kSemThreads + threadIdx.x; q < cells;
         q += (long long)gridDim.x * kSemThreads)
        m = fmaxf(m, e[q]);
    S[threadIdx.x] = m;
    __syncthreads();
    for (int o = kSemThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) S[threadIdx.x] = fmaxf(S[threadIdx.x], S[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax((unsigned int*)&emax[g], __float_as_uint(S[0]));
}

// proj[g][j]: the largest coherence of slowness j over the windows whose
// energy is at least rel_floor * emax[g] (all windows when energy is null);
// -1 when none qualifies.  Grid (np, gathers).
__global__ void __launch_bounds__(kSemThreads)
k_sem_proj(int ntau, const float* __restrict__ coh, const float* __restrict__ energy,
           const float* __restrict__ emax, float rel_floor, float* __restrict__ proj)
{
    __shared__ float S[kSemThreads];
    const int j = blockIdx.x, g = blockIdx.y, np = gridDim.x;
    const long long row = ((long long)g * np + j) * ntau;
    const float fl = energy ? rel_floor * emax[g] : 0.f;
    float m = -1.f;
    for (int i = threadIdx.x; i < ntau; i += kSemThreads)
        if (!energy || energy[row + i] >= fl) m = fmaxf(m, coh[row + i]);
    S[threadIdx.x] = m;
    __syncthreads();
    for (int o = kSemThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) S[threadIdx.x] = fmaxf(S[threadIdx.x], S[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) proj[(long long)g * np + j] = S[0];
}

// The slowness of the largest proj[g][j] among slownesses in [lo, hi] (lo
// raised to ref_scale * p_ref[g] when p_ref is given); ties go to the
// smaller slowness.  One workgroup per gather.
__global__ void __launch_bounds__(kSemThreads)
k_sem_argmax(int np, const float* __restrict__ proj, float p0, float dp,
             const float* __restrict__ p_ref, float ref_scale, float lo, float hi,
             float* __restrict__ p_out, float* __restrict__ c_out)
{
    __shared__ float Sc[kSemThreads];
    __shared__ int Sj[kSemThreads];
    const int g = blockIdx.x;
    const float l = p_ref ? fmaxf(lo, ref_scale * p_ref[g]) : lo;
    float best = -1.f;
    int bj = np;
    for (int j = threadIdx.x; j < np; j += kSemThreads) {
        const float p = p0 + j * dp;
        if (p < l || p > hi) continue;
        const float m = proj[(long long)g * np + j];
        if (m > best) {
            best = m;
            bj = j;
        }
    }
    Sc[threadIdx.x] = best;
    Sj[threadIdx.x] = bj;
    __syncthreads();
    for (int o = kSemThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const float c2 = Sc[threadIdx.x + o];
            const int j2 = Sj[threadIdx.x + o];
            if (c2 > Sc[threadIdx.x] || (c2 == Sc[threadIdx.x] && j2 < Sj[threadIdx.x])) {
                Sc[threadIdx.x] = c2;
                Sj[threadIdx.x] = j2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const bool found = Sj[0] < np && Sc[0] >= 0.f;
        p_out[g] = found ? p0 + Sj[0] * dp : 0.f;
        c_out[g] = found ? Sc[0] : 0.f;
    }
}

__global__ void k_starting_model(int NR, int NZ, float dr, float a, float inv_dist,
                                 const float* __restrict__ vp_wall,
                                 const float* __restrict__ vs_wall,
                                 const float* __restrict__ vp_far, const float* __restrict__ vs_far,
                                 float vp_fluid, float* __restrict__ vp, float* __restrict__ vs)
{
    const long long n = (long long)NR * NZ;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride) {
        const int i = (int)(c / NZ), k = (int)(c % NZ);
        const float r = (i + 0.5f) * dr;
        if (r < a) {
            vp[c] = vp_fluid;
            vs[c] = 0.f;
            continue;
        }
        const float f = fminf((r - a) * inv_dist, 1.f);
        vp[c] = vp_wall[k] + f * (vp_far[k] - vp_wall[k]);
        vs[c] = vs_wall[k] + f * (vs_far[k] - vs_wall[k]);
    }
}

}  // namespace bhfwi

extern "C" {

int bhfwi_semblance(void* stream, int32_t ngather, int32_t nrec, int32_t nt, const float* traces,
                    float dt, const float* offset, int32_t np, float p0, float dp, int32_t ntau,
                    int32_t tau_stride, int32_t win, float* coh, float* energy)
{
    if (ngather < 1 || nrec < 1 || nrec > 64 || nt < 2 || !traces || !offset || !coh ||
        np < 1 || ntau < 1 || tau_stride < 1 || win < 1 || win > bhfwi::kSemSpan ||
        !(dt > 0.f) || ngather > 65535)
        return BHFWI_EINVAL;
    // windows per workgroup: their time range fits the staged span
    const int chunk = (bhfwi::kSemSpan - win) / tau_stride + 1;
    const int nchunk = (ntau + chunk - 1) / chunk;
    if (nchunk > 65535) return BHFWI_EINVAL;
    hipLaunchKernelGGL(bhfwi::k_semblance, dim3(np, ngather, nchunk), dim3(bhfwi::kSemThreads), 0,
                       (hipStream_t)stream, nrec, nt, traces, dt, offset, p0, dp, ntau,
                       tau_stride, win, chunk, coh, energy);
    return hipGetLastError() == hipSuccess ? BHFWI_OK : BHFWI_EHIP;
}

int bhfwi_semblance_pick(void* stream, int32_t ngather, int32_t np, int32_t ntau,
                         const float* coh, const float* energy, float rel_floor, float p0,
                         float dp, const float* p_ref, float ref_scale, float p_lo, float p_hi,
                         float* proj, float* p_out, float* c_out)
{
    if (ngather < 1 || ngather > 65535 || np < 1 || ntau < 1 || !coh || !proj || !p_out ||
        !c_out || !(p_hi >= p_lo) || !(rel_floor >= 0.f))
        return BHFWI_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (energy) {  // c_out holds each gather's largest window energy meanwhile
        hipLaunchKernelGGL(bhfwi::k_sem_fill, dim3((ngather + 255) / 256), dim3(256), 0, st, c_out,
                           ngather, 0.f);
        hipLaunchKernelGGL(bhfwi::k_sem_emax, dim3(64, ngather), dim3(bhfwi::kSemThreads), 0, st,
                           (long long)np * ntau, energy, c_out);
    }
    hipLaunchKernelGGL(bhfwi::k_sem_proj, dim3(np, ngather), dim3(bhfwi::kSemThreads), 0, st,
                       ntau, coh, energy, (const float*)c_out, rel_floor, proj);
    hipLaunchKernelGGL(bhfwi::k_sem_argmax, dim3(ngather), dim3(bhfwi::kSemThreads), 0, st, np,
                       (const float*)proj, p0, dp, p_ref, ref_scale, p_lo, p_hi, p_out, c_out);
    return hipGetLastError() == hipSuccess ? BHFWI_OK : BHFWI_EHIP;
}

int bhfwi_starting_model(void* stream, int32_t NR, int32_t NZ, float dr, float a, float dist,
                         const float* vp_wall, const float* vs_wall, const float* vp_far,
                         const float* vs_far, float vp_fluid, float* vp, float* vs)
{
    if (NR < 1 || NZ < 1 || !(dr > 0.f) || !(dist > 0.f) || !vp_wall || !vs_wall || !vp_far ||
        !vs_far || !vp || !vs)
        return BHFWI_EINVAL;
    const long long n = (long long)NR * NZ;
    const int blocks = (int)std::min<long long>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(bhfwi::k_starting_model, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                       NR, NZ, dr, a, 1.0f / dist, vp_wall, vs_wall, vp_far, vs_far, vp_fluid,
                       vp, vs);
    return hipGetLastError() == hipSuccess ? BHFWI_OK : BHFWI_EHIP;
}

}  // extern "C"
