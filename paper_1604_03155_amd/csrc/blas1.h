// Vector kernels of the Lippmann-Schwinger Bi-CGStab solve (blas1.hip).
#pragma once

#include "common.h"

namespace vg {

// A complex scalar passed by value to the update kernels (rounded to the
// vector precision inside).
struct Cd {
    double re, im;
};

// Dot products sum_i conj(a_j[i]) b_j[i], j < count <= 3.
template <typename R>
struct DotArgs {
    const cplx<R>* a[3];
    const cplx<R>* b[3];
    int count;
};

// Largest number of partial-sum blocks of a reduction: the partial buffer
// holds kDotBlocks * 6 doubles.
constexpr int kDotBlocks = 1024;

template <typename R>
hipError_t ls_post(const void* x, const void* q, void* y, double k2, long long n, hipStream_t s);
template <typename R>
hipError_t ls_rhs(const void* q, const void* phi, void* b, double k2, long long n, hipStream_t s);
template <typename R>
hipError_t axpy(const void* a, Cd alpha, const void* b, void* out, long long n, hipStream_t s);
template <typename R>
hipError_t p_update(const void* r, const void* v, void* p, Cd beta, Cd omega, long long n, hipStream_t s);
template <typename R>
hipError_t xr_update(void* x, void* r, const void* p, const void* sv, const void* t, Cd alpha, Cd omega, long long n,
                     hipStream_t s);
// out[2j], out[2j+1]: real and imaginary part of dot j (device buffer of 6
// doubles); part: device buffer of kDotBlocks * 6 doubles.
template <typename R>
hipError_t dots(const DotArgs<R>& args, double* part, double* out, long long n, hipStream_t s);

}  // namespace vg
