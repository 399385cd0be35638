// Wavefront row operations shared by the 2D row-marching kernels (gfx950):
// one-lane shifts across a wavefront (DPP) and range-checked row stores.
#pragma once
#include <hip/hip_runtime.h>

namespace lbrs {

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Wavefront shifts by one lane (DPP): lane l receives lane l-1 (shr) or
// lane l+1 (shl).  Lanes with no source receive 0 (bound_ctrl, so no
// register needs clearing first) and are halo lanes.
__device__ inline double lane_from_left(double v) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_mov_dpp(lo, 0x138, 0xf, 0xf, true);  // wave_shr:1
    hi = __builtin_amdgcn_mov_dpp(hi, 0x138, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
__device__ inline double lane_from_right(double v) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_mov_dpp(lo, 0x130, 0xf, 0xf, true);  // wave_shl:1
    hi = __builtin_amdgcn_mov_dpp(hi, 0x130, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

// Store one double per lane into one row of one plane; a byte offset voff
// outside [0, row_bytes) is dropped by the buffer range check.
__device__ inline void store_row(double* row, int row_bytes, int voff, double v) {
    __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(row, 0, row_bytes, 0x00020000);
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, 0, 0);
}

}  // namespace lbrs
