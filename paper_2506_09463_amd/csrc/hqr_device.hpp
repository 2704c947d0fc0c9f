// hqr_device.hpp -- device helpers shared by the libhqr kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define HQR_DEV static __device__ __forceinline__

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Column-major element (i, j) with leading dimension ld.
#define HQR_AT(M, i, j, ld) ((M)[(size_t)(i) + (size_t)(j) * (size_t)(ld)])

// Broadcast a double held by lane `src` (wave-uniform) to the whole wave.
HQR_DEV double readlane_f64(double v, int src)
{
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_readlane(lo, src);
    hi = __builtin_amdgcn_readlane(hi, src);
    return __hiloint2double(hi, lo);
}

// Unscaled 2-norm of (x0, tail) is safe when the largest magnitude c lies in
// [2^-460, 2^460]: every square of the largest entries is a normal number and
// a sum of fewer than 2^31 such squares cannot overflow.
HQR_DEV bool norm_fast_path_ok(double c)
{
    return c >= 0x1p-460 && c <= 0x1p460;
}

// Round-to-nearest fp64 -> fp32 conversion.
HQR_DEV float to_f32(double x) { return (float)x; }

// Forces v to be materialized here (empty asm that reads and writes it): a
// load feeding it cannot be sunk into a later conditional block, so a group
// of loads issued before a group of pins waits once for all of them.
HQR_DEV void pin_f64(double &v) { asm volatile("" : "+v"(v)); }
