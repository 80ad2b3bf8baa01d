// bhfwi_internal.h -- device-side shot descriptor shared by the kernels and
// the host code of libbhfwi.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bhfwi {

constexpr int kOwn = 62;  // axial rows owned by one wave64 (lanes 1..62)

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
