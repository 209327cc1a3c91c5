// kct_epilogue.h -- the output epilogues shared by every projector kernel: the
// forward's (p = A x, e = b - A x, the LSQR update of u) and the backward's
// (r = A^T e with the solvers' scalings, Tikhonov term, Jacobi weights, the
// diagonal of A^T A), each returning its contribution to the workgroup's FP64
// partial sum of squares.
#pragma once

#include "kct_internal.h"
#include "kct_weights.h"

namespace kct {

// Store ray `ray` of the forward output from its accumulated value p (already
// multiplied by the ray length factor); returns the square of the stored value.
template <typename TP, int EPI, typename A>
__device__ __forceinline__ double fwd_store(TP *__restrict__ out, const TP *__restrict__ aux,
                                            const Scalars *__restrict__ sc, size_t ray, A p)
{
    A o;
    if (EPI == FWD_BMINUS) o = to_acc(aux[ray]) - p;
    else if (EPI == FWD_LSQR) o = (A)sc->fwd_c1 * p - (A)sc->fwd_c2 * to_acc(out[ray]);
    else if (EPI == FWD_NORM) o = (A)sc->fwd_scale * p;
    else o = p;
    const TP st = store_as<TP>(o);
    out[ray] = st;
    const double od = (double)to_acc(st);
    return od * od;
}

// Store voxel `vox` (z-fastest index vox_z) of the backward output from its
// accumulated value acc; returns its term of the partial sum of squares.
template <typename T, int EPI, typename A>
__device__ __forceinline__ double bwd_store(T *__restrict__ out, T *__restrict__ out_z,
                                            const Scalars *__restrict__ sc, const float *__restrict__ aux,
                                            size_t vox, size_t vox_z, A acc)
{
    A o;
    if (EPI == BWD_LSQR0) o = (A)sc->bwd_c1 * acc;
    else if (EPI == BWD_LSQR) o = (A)sc->bwd_c1 * acc - (A)sc->bwd_c2 * to_acc(out[vox]);
    else if (EPI == BWD_NORM) o = (A)sc->bwd_scale * acc;
    else if (EPI == BWD_TIK) o = (A)sc->bwd_scale * acc - (A)sc->tik_r * (A)aux[vox];
    else if (EPI == BWD_JACOBI) o = (A)aux[vox] * acc;
    else if (EPI == BWD_DIAG_INV) o = acc > 0 ? (A)1 / acc : (A)0;
    else o = acc;
    const T st = store_as<T>(o);
    out[vox] = st;
    if (EPI == BWD_LSQR0 || EPI == BWD_LSQR) out_z[vox_z] = st;
    if (EPI == BWD_JACOBI) {  // |M A^T e|^2 with M^2 = aux: the preconditioned residual norm
        const double a = (double)acc;
        return (double)aux[vox] * a * a;
    }
    const double od = (double)to_acc(st);
    return od * od;
}

// Whether an epilogue writes partial sums.
template <int EPI> constexpr bool bwd_has_partials() { return EPI != BWD_PLAIN && EPI != BWD_DIAG && EPI != BWD_DIAG_INV; }

}  // namespace kct
