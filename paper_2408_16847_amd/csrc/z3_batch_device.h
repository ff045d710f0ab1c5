// Device helpers of the MFMA many-map kernels (forward and adjoint; internal).
#pragma once

#include "z3_device.h"

namespace z3 {

__device__ __forceinline__ int wave_incl_scan(int v, int lane)
{
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int t = __shfl_up(v, o, kWave);
        if (lane >= o) v += t;
    }
    return v;
}

__device__ __forceinline__ int wave_sum_i32(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ float uniform_f32(float x)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// LDS slot of harmonic column c of candidate row r: rows of HS elements (a multiple of 32),
// column bits XOR-swizzled by the row so that both the row-wise writes (one row per lane)
// and the MFMA operand reads (4 rows x 16 columns per instruction) avoid bank conflicts.
template <int HS>
__device__ __forceinline__ int hslot(int r, int c)
{
    const int swz = ((r & 1) << 4) | ((r >> 1) & 15);
    return r * HS + (c ^ swz);
}

// The frame of a wave-uniform pivot, with every field made explicitly wave-uniform.
__device__ __forceinline__ PivotFrame uniform_frame(PivotFrame f)
{
    f.xp = uniform_f64(f.xp); f.yp = uniform_f64(f.yp); f.zp = uniform_f64(f.zp);
    f.th = uniform_f64(f.th); f.sh = uniform_f64(f.sh); f.ch = uniform_f64(f.ch);
    f.inv_sp = uniform_f32(f.inv_sp); f.phf = uniform_f32(f.phf);
    f.nx = uniform_f64(f.nx); f.ny = uniform_f64(f.ny); f.nz = uniform_f64(f.nz);
    f.ex = uniform_f64(f.ex); f.ey = uniform_f64(f.ey);
    return f;
}

}  // namespace z3
