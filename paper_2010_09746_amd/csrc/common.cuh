// Device-side helpers shared by the HIP sources: complex element types, 2x2
// matrices and launch checks.
#pragma once

#include <hip/hip_runtime.h>

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
};

inline void check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        fail(QS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace qsim
