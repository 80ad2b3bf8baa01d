// bhfwi_internal.h -- device-side shot descriptor shared by the kernels and
// the host code of libbhfwi.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bhfwi {

constexpr int kOwn = 62;  // axial rows owned by one wave64 (lanes 1..62)

// Neighbour exchange along the axial direction inside one wave64 (lane =
// axial row): DPP wavefront shifts, no LDS.  Lanes without a source read 0.
__device__ inline float from_lane_below(float v)  // lane l <- lane l - 1
{
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, true));
}
__device__ inline float from_lane_above(float v)  // lane l <- lane l + 1
{
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, true));
}

// Reciprocal within 1 ulp (one v_rcp_f32 instead of a correctly rounded
// division): the medium coefficients and the 1/r factors are set up with it.
__device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// A value that is the same in every lane (it depends on the radial row of
// the wave only) kept in a scalar register.
__device__ inline float wave_uniform(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

// Workgroup b of a launch is dispatched to XCD b % 8.  With map == 1 the n
// workgroups are renumbered so that XCD x walks one contiguous chunk of the
// work table, [x*(n/8) + min(x, n%8), ...), in table order: tiles that are
// neighbours in the table (and share halo rows) then meet in the same L2.
__device__ inline int xcd_chunk(int b, int n, int map)
{
    if (map != 1) return b;
    const int x = b & 7, l = b >> 3, per = n >> 3, rem = n & 7;
    return x * per + min(x, rem) + l;
}

// One shot as the kernels see it.  Offsets are in floats.
struct ShotDev {
    int NR, NZ, nr, nz, pr, pz;
    int nt, src_k, nrec, rec_off;
    float dr, dz, dt, inv_dr, inv_dz, src_scale;
    long long model_off, model_ld;
    long long cell_off;    // offset of this shot's cells in packed per-cell planes
    long long fst_off;     // forward state block within one state buffer
    long long ast_off;     // adjoint state block within one adjoint buffer
    long long trace_off;   // packed traces / residuals
    long long wave_off;    // packed wavelets
    long long psir_len;    // pr * NZ
    long long psiz_len;    // NR * 2 pz
    int pml_r_off, pml_z_off;  // PML coefficient tables
};

}  // namespace bhfwi
