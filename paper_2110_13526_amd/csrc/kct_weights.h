// kct_weights.h -- the one definition of the ray-voxel weight used by both the
// forward projector and the backprojector.
//
// Siddon model (Section 3 of the paper): w_ij is the length of ray i inside
// voxel j.  In the parametrisation of kct_internal.h the part of the ray inside
// voxel (i_xi, i_eta, i_zeta) is the xi-interval
//     [max(lo_xi, lo_eta, lo_zeta), min(hi_xi, hi_eta, hi_zeta)]
// where [lo, hi] on each axis is the xi-range in which the ray is inside that
// axis' cell.  The weight is L * max(0, min(hi) - max(lo)).  min and max are
// exact operations, so any evaluation order of the three lows and highs gives
// the same bits; both kernels compute every low/high with the functions below
// on the same table entries, so they obtain bitwise identical xi-lengths.  L is
// one bitwise identical number per ray: the forward kernel multiplies the
// ray's sum by it, the backprojector multiplies the projection value by it.
//
// A ray parallel to the planes of an axis (a = 0 or qz = 0) is inside the one
// cell floor(c + h) of that axis (cells are half-open [lo, hi); plane m of the
// axis is at m - h in its index frame, see kct_internal.h), over the whole xi
// range.
//
// Floating-point contraction is switched off here: fused multiply-adds could
// otherwise round the same expression differently in the two kernels.
#pragma once

#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kct_internal.h"

namespace kct {

// xi at which the ray crosses the plane mb (index frame) of an axis whose
// coordinate along the ray is c + xi / inv.
__host__ __device__ __forceinline__ float cross_at(float mb, float c, float inv) { return (mb - c) * inv; }

// zeta of the ray at xi = 0 (one rounding), and d xi / d zeta.
__host__ __device__ __forceinline__ float zeta_centre(float qz, float tcv, float zc)
{
    return __builtin_fmaf(qz, tcv, -zc);
}
__host__ __device__ __forceinline__ float zeta_inv_slope(float inv_qz, float kz) { return inv_qz * kz; }

// xi at which a ray crosses the zeta-plane h (index frame), from the ray's
// offset nzc = zeta_offset(zeta_c, czr): one fused multiply-add per plane.
// The forward's z-walk and the backprojector's candidates take every zeta
// crossing from these two, so both see the same bits.
__host__ __device__ __forceinline__ float zeta_offset(float zc, float czr) { return -(zc * czr); }
__host__ __device__ __forceinline__ float zeta_cross(float h, float nzc, float czr) { return __builtin_fmaf(h, czr, nzc); }

// Length of the ray in mm per unit of xi.  On the GPU the hardware square root
// (within 1 ulp; one instruction instead of the correctly rounded sequence):
// every kernel takes L from this function, so L stays one number per ray.
__host__ __device__ __forceinline__ float ray_length_per_xi(float lxy2, float qz, float gp)
{
    float t = qz * gp;
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_sqrtf(lxy2 + t * t);
#else
    return sqrtf(lxy2 + t * t);
#endif
}

// The cell (0-based) that a ray parallel to an axis' planes lies in (h: the
// axis' plane offset).
__host__ __device__ __forceinline__ int parallel_cell(float c, float h) { return (int)floorf(c + h); }

// xi-range [lo, hi] of cell m of an axis with plane offset half_n (plane m at
// m - half_n), for a ray whose coordinate on that axis is c + xi / inv (inv ==
// 0: parallel).  mb must be the cell's lower plane, (float)m - half_n (exact:
// half_n is a multiple of 1/2), passed in so callers that walk consecutive
// cells need not recompute it.
__host__ __device__ __forceinline__ void cell_range_mb(int m, float mb, float half_n, float c, float inv, float &lo,
                                                       float &hi)
{
    if (inv == 0.0f) {
        bool in = (m == parallel_cell(c, half_n));
        lo = in ? -INFINITY : INFINITY;
        hi = INFINITY;
    } else {
        float b0 = cross_at(mb, c, inv);
        float b1 = cross_at(mb + 1.0f, c, inv);
        lo = fminf(b0, b1);
        hi = fmaxf(b0, b1);
    }
}

__host__ __device__ __forceinline__ void cell_range(int m, float half_n, float c, float inv, float &lo, float &hi)
{
    cell_range_mb(m, (float)m - half_n, half_n, c, inv, lo, hi);
}

// ---------------------------------------------------------------- storage

// Storage types: float, bfloat16 (raw bits, round-to-nearest-even on store,
// see kct_internal.h) and IEEE half.  Arithmetic is always single precision.

__host__ __device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(bf16 v) { return __uint_as_float(((uint32_t)v.bits) << 16); }
__device__ __forceinline__ float to_f32(_Float16 v) { return (float)v; }

template <typename T> __device__ __forceinline__ T from_f32(float v);
template <> __device__ __forceinline__ float from_f32<float>(float v) { return v; }
template <> __device__ __forceinline__ bf16 from_f32<bf16>(float v)
{
    uint32_t u = __float_as_uint(v);
    bf16 r;
    if ((u & 0x7fffffffu) > 0x7f800000u) {  // NaN stays NaN
        r.bits = (uint16_t)((u >> 16) | 0x40u);
        return r;
    }
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest, ties to even
    r.bits = (uint16_t)(u >> 16);
    return r;
}
template <> __device__ __forceinline__ _Float16 from_f32<_Float16>(float v) { return (_Float16)v; }

// Accumulator type of a storage type: single precision for the 32- and 16-bit
// types; double for double storage, which exists so that the projector pair
// can be evaluated to double-precision rounding (gradient checks).  The
// weights are the same single-precision numbers in every case.
template <typename T> struct acc_of { using type = float; };
template <> struct acc_of<double> { using type = double; };
template <typename T> using acc_t = typename acc_of<T>::type;

__host__ __device__ __forceinline__ float to_acc(float v) { return v; }
__device__ __forceinline__ float to_acc(bf16 v) { return to_f32(v); }
__device__ __forceinline__ float to_acc(_Float16 v) { return (float)v; }
__host__ __device__ __forceinline__ double to_acc(double v) { return v; }

template <typename T> __device__ __forceinline__ T store_as(acc_t<T> v) { return from_f32<T>(v); }
template <> __device__ __forceinline__ double store_as<double>(double v) { return v; }

// acc + w * v with one rounding, in the accumulator's precision.
__host__ __device__ __forceinline__ float fma_acc(float w, float v, float acc) { return __builtin_fmaf(w, v, acc); }
__host__ __device__ __forceinline__ double fma_acc(float w, double v, double acc)
{
    return __builtin_fma((double)w, v, acc);
}

}  // namespace kct
