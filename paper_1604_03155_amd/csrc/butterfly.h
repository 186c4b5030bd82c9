// Small DFT kernels ("butterflies") of radix 2, 3, 4, 5, 7, 8, 16 and 32 used
// by the Stockham FFT passes.  DIR = -1 computes y_m = sum_r v_r e^{-2 pi i r m / R}
// (forward), DIR = +1 the conjugate-exponent sum (inverse, unnormalised).
#pragma once

#include <utility>

#include "common.h"

namespace vg {

// v * (DIR * i)
template <int DIR, typename R>
__device__ __forceinline__ cplx<R> mul_diri(cplx<R> v) {
    return DIR < 0 ? mk(v.y, -v.x) : mk(-v.y, v.x);
}

template <int DIR, typename R>
__device__ __forceinline__ void dft2(cplx<R>& a, cplx<R>& b) {
    cplx<R> t = a - b;
    a = a + b;
    b = t;
}

template <int DIR, typename R>
__device__ __forceinline__ void dft4(cplx<R>& v0, cplx<R>& v1, cplx<R>& v2, cplx<R>& v3) {
    cplx<R> s02 = v0 + v2, d02 = v0 - v2;
    cplx<R> s13 = v1 + v3, d13 = mul_diri<DIR>(v1 - v3);
    v0 = s02 + s13;
    v2 = s02 - s13;
    v1 = d02 + d13;
    v3 = d02 - d13;
}

template <int DIR, typename R>
__device__ __forceinline__ void dft8(cplx<R>* v) {
    // even / odd halves, then combine with W8^m = e^{DIR i pi m / 4}
    dft4<DIR>(v[0], v[2], v[4], v[6]);
    dft4<DIR>(v[1], v[3], v[5], v[7]);
    const R h = R(0.70710678118654752440);
    cplx<R> o1 = mk(h * (v[3].x - DIR * v[3].y), h * (v[3].y + DIR * v[3].x));
    cplx<R> o2 = mul_diri<DIR>(v[5]);
    cplx<R> o3 = mk(h * (-v[7].x - DIR * v[7].y), h * (-v[7].y + DIR * v[7].x));
    cplx<R> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    cplx<R> o0 = v[1];
    v[0] = e0 + o0;
    v[4] = e0 - o0;
    v[1] = e1 + o1;
    v[5] = e1 - o1;
    v[2] = e2 + o2;
    v[6] = e2 - o2;
    v[3] = e3 + o3;
    v[7] = e3 - o3;
}

template <int DIR, typename R>
__device__ __forceinline__ void dft3(cplx<R>* v) {
    const R s3 = R(0.86602540378443864676);
    cplx<R> t = v[1] + v[2];
    cplx<R> u = mul_diri<DIR>(v[1] - v[2]);
    cplx<R> m = v[0] - scale(t, R(0.5));
    v[0] = v[0] + t;
    v[1] = m + scale(u, s3);
    v[2] = m - scale(u, s3);
}

// Odd prime radix by pairing r with R - r:
//   y_m = v_0 + sum_{r=1}^{(R-1)/2} [(v_r + v_{R-r}) cos(2 pi r m/R)
//                                     + DIR i (v_r - v_{R-r}) sin(2 pi r m/R)]
template <int RAD, int DIR, typename R>
__device__ __forceinline__ void dft_odd(cplx<R>* v, const double* cs, const double* sn) {
    constexpr int H = (RAD - 1) / 2;
    cplx<R> a[H], b[H];
#pragma unroll
    for (int r = 1; r <= H; ++r) {
        a[r - 1] = v[r] + v[RAD - r];
        b[r - 1] = mul_diri<DIR>(v[r] - v[RAD - r]);
    }
    cplx<R> y[RAD];
    cplx<R> s0 = v[0];
#pragma unroll
    for (int r = 0; r < H; ++r) s0 = s0 + a[r];
    y[0] = s0;
#pragma unroll
    for (int m = 1; m <= H; ++m) {
        cplx<R> re = v[0], im = mk(R(0), R(0));
#pragma unroll
        for (int r = 1; r <= H; ++r) {
            const int idx = (r * m) % RAD;  // in [1, RAD-1]
            const R c = R(cs[idx <= H ? idx : RAD - idx]);
            const R s = R(idx <= H ? sn[idx] : -sn[RAD - idx]);
            re = re + scale(a[r - 1], c);
            im = im + scale(b[r - 1], s);
        }
        y[m] = re + im;
        y[RAD - m] = re - im;
    }
#pragma unroll
    for (int m = 0; m < RAD; ++m) v[m] = y[m];
}

template <int DIR, typename R>
__device__ __forceinline__ void dft5(cplx<R>* v) {
    // cos and sin of 2 pi j / 5, j = 0..2
    constexpr double cs[3] = {1.0, 0.30901699437494742410, -0.80901699437494742410};
    constexpr double sn[3] = {0.0, 0.95105651629515357212, 0.58778525229247312917};
    dft_odd<5, DIR>(v, cs, sn);
}

template <int DIR, typename R>
__device__ __forceinline__ void dft7(cplx<R>* v) {
    // cos and sin of 2 pi j / 7, j = 0..3
    constexpr double cs[4] = {1.0, 0.62348980185873353053, -0.22252093395631440429,
                              -0.90096886790241912624};
    constexpr double sn[4] = {0.0, 0.78183148246802980871, 0.97492791218182360702,
                              0.43388373911755812048};
    dft_odd<7, DIR>(v, cs, sn);
}

// Runtime radix dispatch (v holds at least `radix` values).
template <int DIR, typename R>
__device__ __forceinline__ void dft_any(int radix, cplx<R>* v) {
    switch (radix) {
        case 2: dft2<DIR>(v[0], v[1]); break;
        case 3: dft3<DIR>(v); break;
        case 4: dft4<DIR>(v[0], v[1], v[2], v[3]); break;
        case 5: dft5<DIR>(v); break;
        case 7: dft7<DIR>(v); break;
        default: dft8<DIR>(v); break;
    }
}

// ------------------------------------------------ radix 16 and 32 --------
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    [&]<int... I>(std::integer_sequence<int, I...>) { (f(std::integral_constant<int, I>{}), ...); }
    (std::make_integer_sequence<int, N>{});
}

// cos(2 pi k / 32) for k = 0..8; other angles follow by symmetry.
constexpr double kCos32[9] = {1.0,
                              0.98078528040323044912618,
                              0.92387953251128675612818,
                              0.83146961230254523707879,
                              0.70710678118654752440084,
                              0.55557023301960222474283,
                              0.38268343236508977172846,
                              0.19509032201612826784828,
                              0.0};

constexpr double cos32(int k) {
    k = ((k % 32) + 32) % 32;
    if (k <= 8) return kCos32[k];
    if (k <= 16) return -kCos32[16 - k];
    if (k <= 24) return -kCos32[k - 16];
    return kCos32[32 - k];
}
constexpr double sin32(int k) { return cos32(k - 8); }

// v * e^{DIR 2 pi i m / RR} for a compile-time m (RR divides 32); the four
// axis-aligned cases cost no multiplications.
template <int RR, int m, int DIR, typename R>
__device__ __forceinline__ cplx<R> wmul_const(cplx<R> v) {
    constexpr int mm = ((m % RR) + RR) % RR;
    if constexpr (mm == 0) {
        return v;
    } else if constexpr (4 * mm == RR) {
        return mul_diri<DIR>(v);
    } else if constexpr (2 * mm == RR) {
        return mk(-v.x, -v.y);
    } else if constexpr (4 * mm == 3 * RR) {
        return mul_diri<-DIR>(v);
    } else {
        constexpr int k = mm * (32 / RR);
        constexpr R c = R(cos32(k));
        constexpr R sn = R(DIR * sin32(k));
        return mk(v.x * c - v.y * sn, v.y * c + v.x * sn);
    }
}

template <int RAD, int DIR, typename R>
__device__ __forceinline__ void dft_fixed(cplx<R>* v);

// DFT of size R1*R2 in registers (Cooley-Tukey): R1 DFTs of size R2 over
// stride-R1 subsequences, twiddles W_{R1 R2}^{n1 k2}, R2 DFTs of size R1;
// output index k2 + R2 k1.
template <int R1, int R2, int DIR, typename R>
__device__ __forceinline__ void dft_ct(cplx<R>* v) {
    constexpr int RR = R1 * R2;
    cplx<R> a[RR];
    static_for<R1>([&](auto n1c) {
        constexpr int n1 = decltype(n1c)::value;
        cplx<R> s[R2];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) s[n2] = v[n1 + R1 * n2];
        dft_fixed<R2, DIR>(s);
        static_for<R2>([&](auto k2c) {
            constexpr int k2 = decltype(k2c)::value;
            a[n1 * R2 + k2] = wmul_const<RR, n1 * k2, DIR>(s[k2]);
        });
    });
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) {
        cplx<R> s[R1];
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) s[n1] = a[n1 * R2 + k2];
        dft_fixed<R1, DIR>(s);
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) v[k2 + R2 * k1] = s[k1];
    }
}

// Compile-time radix dispatch.
template <int RAD, int DIR, typename R>
__device__ __forceinline__ void dft_fixed(cplx<R>* v) {
    if constexpr (RAD == 2) dft2<DIR>(v[0], v[1]);
    else if constexpr (RAD == 3) dft3<DIR>(v);
    else if constexpr (RAD == 4) dft4<DIR>(v[0], v[1], v[2], v[3]);
    else if constexpr (RAD == 5) dft5<DIR>(v);
    else if constexpr (RAD == 7) dft7<DIR>(v);
    else if constexpr (RAD == 8) dft8<DIR>(v);
    else if constexpr (RAD == 16) dft_ct<4, 4, DIR>(v);
    else if constexpr (RAD == 32) dft_ct<4, 8, DIR>(v);
    else static_assert(RAD == 2, "unsupported radix");
}

}  // namespace vg
