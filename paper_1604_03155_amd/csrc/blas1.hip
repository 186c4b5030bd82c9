// Vector kernels of the Bi-CGStab solve of the Lippmann-Schwinger equation
// (Section 5.3): fused updates and multi-dot reductions over complex vectors
// of the plan's precision, with dot products accumulated in FP64.
#include "common.h"
#include "blas1.h"

namespace vg {

namespace {

constexpr int kBlock = 256;

template <typename R>
__device__ __forceinline__ cplx<R> cfrom(const Cd& a) {
    return mk((R)a.re, (R)a.im);
}

// y = -x + k2 * q .* y  (the Lippmann-Schwinger operator after y = T * x)
template <typename R>
__global__ void __launch_bounds__(kBlock) ls_post_kernel(const cplx<R>* __restrict__ x, const cplx<R>* __restrict__ q,
                                                         cplx<R>* __restrict__ y, R k2, long long n) {
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
        const cplx<R> qy = cmul(q[i], y[i]);
        y[i] = mk(k2 * qy.x - x[i].x, k2 * qy.y - x[i].y);
    }
}

// b = -k2 * q .* phi_in
template <typename R>
__global__ void __launch_bounds__(kBlock) ls_rhs_kernel(const cplx<R>* __restrict__ q, const cplx<R>* __restrict__ phi,
                                                        cplx<R>* __restrict__ b, R k2, long long n) {
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
        const cplx<R> v = cmul(q[i], phi[i]);
        b[i] = mk(-k2 * v.x, -k2 * v.y);
    }
}

// out = a + alpha * b (out may alias a)
template <typename R>
__global__ void __launch_bounds__(kBlock) axpy_kernel(const cplx<R>* a, Cd alpha, const cplx<R>* __restrict__ b,
                                                      cplx<R>* out, long long n) {
    const cplx<R> al = cfrom<R>(alpha);
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
        out[i] = a[i] + cmul(al, b[i]);
}

// p = r + beta * (p - omega * v)
template <typename R>
__global__ void __launch_bounds__(kBlock) p_update_kernel(const cplx<R>* __restrict__ r, const cplx<R>* __restrict__ v,
                                                          cplx<R>* __restrict__ p, Cd beta, Cd omega, long long n) {
    const cplx<R> be = cfrom<R>(beta), om = cfrom<R>(omega);
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
        p[i] = r[i] + cmul(be, p[i] - cmul(om, v[i]));
}

// x += alpha * p + omega * s;  r = s - omega * t
template <typename R>
__global__ void __launch_bounds__(kBlock) xr_update_kernel(cplx<R>* __restrict__ x, cplx<R>* __restrict__ r,
                                                           const cplx<R>* __restrict__ p, const cplx<R>* __restrict__ s,
                                                           const cplx<R>* __restrict__ t, Cd alpha, Cd omega,
                                                           long long n) {
    const cplx<R> al = cfrom<R>(alpha), om = cfrom<R>(omega);
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
        const cplx<R> si = s[i];
        x[i] = x[i] + cmul(al, p[i]) + cmul(om, si);
        r[i] = si - cmul(om, t[i]);
    }
}

// Up to 3 dot products sum_i conj(a_j[i]) b_j[i] at once: per-block partial
// sums in FP64 (LDS tree), written to part[block][j].
template <typename R>
__global__ void __launch_bounds__(kBlock) dots_kernel(DotArgs<R> args, double* __restrict__ part, long long n) {
    __shared__ double red[2 * 3][kBlock];
    double acc[2 * 3] = {0, 0, 0, 0, 0, 0};
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            if (j < args.count) {
                const cplx<R> a = args.a[j][i], b = args.b[j][i];
                acc[2 * j] += (double)a.x * b.x + (double)a.y * b.y;
                acc[2 * j + 1] += (double)a.x * b.y - (double)a.y * b.x;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 6; ++j) red[j][threadIdx.x] = acc[j];
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int j = 0; j < 6; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[(long long)blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// Sum of the per-block partials in block order (deterministic): out[6].
__global__ void __launch_bounds__(kBlock) dots_final_kernel(const double* __restrict__ part, int nblocks,
                                                           double* __restrict__ out) {
    __shared__ double red[6][kBlock];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += kBlock)
#pragma unroll
        for (int j = 0; j < 6; ++j) acc[j] += part[(long long)b * 6 + j];
#pragma unroll
    for (int j = 0; j < 6; ++j) red[j][threadIdx.x] = acc[j];
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int j = 0; j < 6; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) out[threadIdx.x] = red[threadIdx.x][0];
}

unsigned grid_for(long long n) {
    const long long b = (n + kBlock * 8 - 1) / (kBlock * 8);
    return (unsigned)(b < 1 ? 1 : (b > kDotBlocks ? kDotBlocks : b));
}

}  // namespace

template <typename R>
hipError_t ls_post(const void* x, const void* q, void* y, double k2, long long n, hipStream_t s) {
    hipLaunchKernelGGL(ls_post_kernel<R>, dim3(grid_for(n)), dim3(kBlock), 0, s, (const cplx<R>*)x, (const cplx<R>*)q,
                       (cplx<R>*)y, (R)k2, n);
    return hipGetLastError();
}

template <typename R>
hipError_t ls_rhs(const void* q, const void* phi, void* b, double k2, long long n, hipStream_t s) {
    hipLaunchKernelGGL(ls_rhs_kernel<R>, dim3(grid_for(n)), dim3(kBlock), 0, s, (const cplx<R>*)q,
                       (const cplx<R>*)phi, (cplx<R>*)b, (R)k2, n);
    return hipGetLastError();
}

template <typename R>
hipError_t axpy(const void* a, Cd alpha, const void* b, void* out, long long n, hipStream_t s) {
    hipLaunchKernelGGL(axpy_kernel<R>, dim3(grid_for(n)), dim3(kBlock), 0, s, (const cplx<R>*)a, alpha,
                       (const cplx<R>*)b, (cplx<R>*)out, n);
    return hipGetLastError();
}

template <typename R>
hipError_t p_update(const void* r, const void* v, void* p, Cd beta, Cd omega, long long n, hipStream_t s) {
    hipLaunchKernelGGL(p_update_kernel<R>, dim3(grid_for(n)), dim3(kBlock), 0, s, (const cplx<R>*)r,
                       (const cplx<R>*)v, (cplx<R>*)p, beta, omega, n);
    return hipGetLastError();
}

template <typename R>
hipError_t xr_update(void* x, void* r, const void* p, const void* sv, const void* t, Cd alpha, Cd omega, long long n,
                     hipStream_t s) {
    hipLaunchKernelGGL(xr_update_kernel<R>, dim3(grid_for(n)), dim3(kBlock), 0, s, (cplx<R>*)x, (cplx<R>*)r,
                       (const cplx<R>*)p, (const cplx<R>*)sv, (const cplx<R>*)t, alpha, omega, n);
    return hipGetLastError();
}

template <typename R>
hipError_t dots(const DotArgs<R>& args, double* part, double* out, long long n, hipStream_t s) {
    const unsigned g = grid_for(n);
    hipLaunchKernelGGL(dots_kernel<R>, dim3(g), dim3(kBlock), 0, s, args, part, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(dots_final_kernel, dim3(1), dim3(kBlock), 0, s, (const double*)part, (int)g, out);
    return hipGetLastError();
}

#define VG_BLAS1_INSTANTIATE(R)                                                                              \
    template hipError_t ls_post<R>(const void*, const void*, void*, double, long long, hipStream_t);        \
    template hipError_t ls_rhs<R>(const void*, const void*, void*, double, long long, hipStream_t);         \
    template hipError_t axpy<R>(const void*, Cd, const void*, void*, long long, hipStream_t);              \
    template hipError_t p_update<R>(const void*, const void*, void*, Cd, Cd, long long, hipStream_t);      \
    template hipError_t xr_update<R>(void*, void*, const void*, const void*, const void*, Cd, Cd, long long, \
                                     hipStream_t);                                                           \
    template hipError_t dots<R>(const DotArgs<R>&, double*, double*, long long, hipStream_t);
VG_BLAS1_INSTANTIATE(float)
VG_BLAS1_INSTANTIATE(double)

}  // namespace vg
