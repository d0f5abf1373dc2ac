// Device-side helpers shared by the HIP sources: complex element types, 2x2
// matrices and launch checks.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "internal.h"

namespace qsim {

// A complex amplitude: plain aggregate (re, im), aligned to its size so that
// one amplitude moves with one 8- or 16-byte access.
template <typename R> struct alignas(2 * sizeof(R)) Cplx {
    R x, y;
};
template <typename R> struct Cx {
    using T = Cplx<R>;
};

// fused multiply-add in the amplitude's own precision
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// 2x2 complex matrix, row-major (u00, u01, u10, u11) as re/im pairs.
template <typename R> struct Mat {
    R a[8];
    Mat() = default;
    __host__ explicit Mat(const double *u)
    {
        for (int i = 0; i < 8; ++i)
            a[i] = (R)u[i];
    }
    // m00 x + m01 y
    template <typename C> __device__ __forceinline__ C row0(C x, C y) const
    {
        C r;
        r.x = a[0] * x.x - a[1] * x.y + a[2] * y.x - a[3] * y.y;
        r.y = a[0] * x.y + a[1] * x.x + a[2] * y.y + a[3] * y.x;
        return r;
    }
    // m10 x + m11 y
    template <typename C> __device__ __forceinline__ C row1(C x, C y) const
    {
        C r;
        r.x = a[4] * x.x - a[5] * x.y + a[6] * y.x - a[7] * y.y;
        r.y = a[4] * x.y + a[5] * x.x + a[6] * y.y + a[7] * y.x;
        return r;
    }
    // (x, y) <- (m00 x + m01 y, m10 x + m11 y), updated in place.  The terms
    // in x are summed first, so x is dead before the new x is written and only
    // one value needs a temporary.
    template <typename C> __device__ __forceinline__ void apply(C &x, C &y) const
    {
        R t0 = a[0] * x.x, t1 = a[0] * x.y, t2 = a[4] * x.x, t3 = a[4] * x.y;
        t0 = fmadd(-a[1], x.y, t0);
        t1 = fmadd(a[1], x.x, t1);
        t2 = fmadd(-a[5], x.y, t2);
        t3 = fmadd(a[5], x.x, t3);
        t0 = fmadd(a[2], y.x, t0);
        t1 = fmadd(a[2], y.y, t1);
        t2 = fmadd(a[6], y.x, t2);
        t3 = fmadd(a[6], y.y, t3);
        x.x = fmadd(-a[3], y.y, t0);
        x.y = fmadd(a[3], y.x, t1);
        const R ny = fmadd(-a[7], y.y, t2);
        y.y = fmadd(a[7], y.x, t3);
        y.x = ny;
    }
};

inline void check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        fail(QS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace qsim
