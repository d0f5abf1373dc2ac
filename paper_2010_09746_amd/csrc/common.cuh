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
    // (x, y) <- (m00 x + m01 y, m10 x + m11 y), updated in place.  Each output
    // first sums the three terms that do not read its own old value; the
    // last term reads the output's own register, so every result lands where
    // its input was and no copies are needed.
    template <typename C> __device__ __forceinline__ void apply(C &x, C &y) const
    {
        R p0 = -a[1] * x.y, p1 = a[1] * x.x, p2 = a[4] * x.x, p3 = a[4] * x.y;
        p0 = fmadd(a[2], y.x, p0);
        p1 = fmadd(a[2], y.y, p1);
        p2 = fmadd(-a[5], x.y, p2);
        p3 = fmadd(a[5], x.x, p3);
        p0 = fmadd(-a[3], y.y, p0);
        p1 = fmadd(a[3], y.x, p1);
        p2 = fmadd(-a[7], y.y, p2);
        p3 = fmadd(a[7], y.x, p3);
        x.x = fmadd(a[0], x.x, p0);
        x.y = fmadd(a[0], x.y, p1);
        y.x = fmadd(a[6], y.x, p2);
        y.y = fmadd(a[6], y.y, p3);
    }
};

// Streaming access to one amplitude: non-temporal loads and stores, for
// kernels that read and write each amplitude once per launch over a state far
// larger than the caches.
template <typename C> __device__ __forceinline__ C ld_stream(const C *p)
{
    C v;
    v.x = __builtin_nontemporal_load(&p->x);
    v.y = __builtin_nontemporal_load(&p->y);
    return v;
}
template <typename C> __device__ __forceinline__ void st_stream(C *p, const C &v)
{
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
}

inline void check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        fail(QS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace qsim
