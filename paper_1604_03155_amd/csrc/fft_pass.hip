// Batched 1D FFT passes over one axis of a strided 2D/3D array, with the
// convolution's padding, kernel multiply, derivative multiply and cropping
// fused in (Section 4's aperiodic convolution: zero padding to 2N per axis,
// forward FFT, multiplication by the spectrum of T, inverse FFT, crop).
//
// Algorithm: Stockham autosort FFT.  With L = R_0 R_1 ... R_{S-1} and Ns the
// product of the radices already done, stage s processes butterflies
// j in [0, L/R): it reads v_r = x[j + r L/R], multiplies v_r by the twiddle
// W_L^{r (j mod Ns) L/(Ns R)}, takes a radix-R DFT, and writes y_r to
// index (j div Ns) Ns R + (j mod Ns) + r Ns.  After the last stage the output
// is in natural order.
//
// Workgroup = C pencils of length L.  The first stage reads global memory
// directly (zero-padded entries e >= n_in are never loaded), intermediate
// stages ping-pong through LDS, and the last stage writes global memory
// directly (entries e >= n_out are never stored).  In column passes lanes map
// to adjacent pencils, so every global access is a run of C adjacent
// elements; in row passes lanes map to adjacent elements of one pencil.
#include "common.h"
#include "butterfly.h"

namespace vg {

namespace {

enum Src : int { SRC_GLOBAL = 0, SRC_LDS = 1 };
enum Dst : int { DST_LDS = 0, DST_GLOBAL = 1, DST_TABLE = 2 };

struct Tile {
    long long in_base0, out_base0;  // address of pencil q = 0
    long long in_qstride, out_qstride;
    int nvalid;                     // pencils of this tile that exist
    int col0;                       // first column (column passes)
    long long o;                    // outer index (column passes)
};

template <int MODE>
__device__ __forceinline__ int lidx(int q, int e, int C, int L) {
    return MODE == MODE_COL ? e * C + q : q * L + e;
}

template <int MODE>
__device__ __forceinline__ Tile make_tile(const PassDesc& p) {
    Tile t;
    if (MODE == MODE_COL) {
        const int ntile = (p.inner + p.C - 1) / p.C;
        const long long o = blockIdx.x / ntile;
        const int c0 = (blockIdx.x % ntile) * p.C;
        t.in_base0 = o * p.in_so + c0;
        t.out_base0 = o * p.out_so + c0;
        t.in_qstride = 1;
        t.out_qstride = 1;
        t.nvalid = min(p.C, p.inner - c0);
        t.col0 = c0;
        t.o = o;
    } else {
        const long long o0 = (long long)blockIdx.x * p.C;
        t.in_base0 = o0 * p.in_so;
        t.out_base0 = o0 * p.out_so;
        t.in_qstride = p.in_so;
        t.out_qstride = p.out_so;
        t.nvalid = (int)min((long long)p.C, (long long)p.outer - o0);
        t.col0 = 0;
        t.o = 0;
    }
    return t;
}

// signed frequency of index e on an L-point DFT, 0 at the Nyquist index
__device__ __forceinline__ int signed_freq(int e, int L) {
    const int h = L >> 1;
    return e < h ? e : (e == h && !(L & 1) ? 0 : e - L);
}

// Length of the whole axis and the spectral index along it of output e of a
// pencil with outer index o (four-step passes map (o, e) to o + L1 e).
__device__ __forceinline__ int axis_len(const PassDesc& p) { return p.L_big ? p.L_big : p.L; }
__device__ __forceinline__ int axis_index(const PassDesc& p, int e, long long o) {
    return p.fs_L1 ? (int)(o + (long long)p.fs_L1 * e) : e;
}

template <typename R>
__device__ __forceinline__ cplx<R> times_ikappa(cplx<R> v, int k, int L, double kscale) {
    const R kap = R(kscale * (double)signed_freq(k, L));
    return mk(-kap * v.y, kap * v.x);
}

template <typename R>
__device__ __forceinline__ cplx<R> table_value(const PassDesc& p, int e, int col, long long o) {
    const int L = axis_len(p);
    const int k = axis_index(p, e, o);
    if (p.table_full) {
        // every spectral index stored: flat = k L^(d-1) + column
        const long long plane = p.d == 3 ? (long long)L * L : (long long)L;
        return reinterpret_cast<const cplx<R>*>(p.table)[(long long)k * plane + col];
    }
    const int N1 = p.tabN + 1;
    const int f1 = min(k, L - k);
    long long flat;
    if (p.d == 3) {
        const int k2 = col / L, k3 = col - (col / L) * L;
        flat = ((long long)f1 * N1 + min(k2, L - k2)) * p.tab_pitch + min(k3, L - k3);
    } else {
        flat = (long long)f1 * N1 + min(col, L - col);
    }
    if (p.table_complex) return reinterpret_cast<const cplx<R>*>(p.table)[flat];
    return mk(reinterpret_cast<const R*>(p.table)[flat], R(0));
}

// four-step twiddle W_{L_big}^{o e} (post_tw == 1) or its conjugate (2)
template <typename R>
__device__ __forceinline__ cplx<R> post_twiddle(const PassDesc& p, cplx<R> v, int e, long long o) {
    const long long idx = (o * (long long)e) % p.L_big;
    const cplx<R> w = reinterpret_cast<const cplx<R>*>(p.tw_big)[idx];
    return p.post_tw == 1 ? cmul(v, w) : cmulc(v, w);
}

// One run of S Stockham stages.
//   src_kind == SRC_GLOBAL: stage 0 reads gsrc (entries e >= n_in read as 0);
//   src_kind == SRC_LDS:    stage 0 reads LDS buffer lsrc.
// Intermediate stages ping-pong between lsrc and lwork.  The last stage
//   DST_GLOBAL: stores entries e < n_out to gdst;
//   DST_TABLE:  multiplies by the Khat octant and stores to LDS buffer tabdst
//               (which must differ from lsrc and lwork).
// deriv_in multiplies the global input by i*kappa(e); rawdst (optional) receives
// i*kappa(e) times the global input, for a second run.
template <typename R, int MODE, int DIR>
__device__ void run_fft(const PassDesc& p, const Tile& t, int src_kind, const cplx<R>* gsrc,
                        cplx<R>* lsrc, cplx<R>* lwork, int dst_kind, cplx<R>* gdst,
                        cplx<R>* tabdst, bool deriv_in, cplx<R>* rawdst) {
    const int L = p.L, C = p.C, S = p.nst;
    const int tid = threadIdx.x, NT = blockDim.x;
    const cplx<R>* tw = reinterpret_cast<const cplx<R>*>(p.tw);
    cplx<R>* seq[2] = {lsrc, lwork};
    const int wsel = (src_kind == SRC_GLOBAL) ? 0 : 1;
    int Ns = 1;
    for (int s = 0; s < S; ++s) {
        const int Rr = p.radix[s];
        const int LR = L / Rr;
        const int nb = C * LR;
        const bool gload = (s == 0 && src_kind == SRC_GLOBAL);
        const bool last = (s == S - 1);
        const cplx<R>* in_l = seq[(s + wsel + 1) & 1];
        cplx<R>* out_l = (last && dst_kind == DST_TABLE) ? tabdst : seq[(s + wsel) & 1];
        const int stw = (Ns > 1) ? L / (Ns * Rr) : 0;
        cplx<R> v[8];
        for (int b = tid; b < nb; b += NT) {
            int q, j;
            if (MODE == MODE_COL) {
                q = b % C;
                j = b / C;
            } else {
                j = b % LR;
                q = b / LR;
            }
            const bool qok = q < t.nvalid;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                if (r < Rr) {
                    const int e = j + r * LR;
                    cplx<R> x;
                    if (gload) {
                        x = mk(R(0), R(0));
                        if (qok && e < p.n_in) x = gsrc[t.in_base0 + q * t.in_qstride + (long long)e * p.in_se];
                        if (rawdst || deriv_in) {
                            const cplx<R> dx = times_ikappa(x, axis_index(p, e, t.o), axis_len(p), p.kscale);
                            if (rawdst) rawdst[lidx<MODE>(q, e, C, L)] = dx;
                            if (deriv_in) x = dx;
                        }
                    } else {
                        x = in_l[lidx<MODE>(q, e, C, L)];
                    }
                    v[r] = x;
                }
            }
            if (Ns > 1) {
                const int k = j % Ns;
#pragma unroll
                for (int r = 1; r < 8; ++r) {
                    if (r < Rr) {
                        const cplx<R> w = tw[r * k * stw];
                        v[r] = DIR < 0 ? cmul(v[r], w) : cmulc(v[r], w);
                    }
                }
            }
            dft_any<DIR>(Rr, v);
            const int ob = (j / Ns) * Ns * Rr + (j % Ns);
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                if (r < Rr) {
                    const int e = ob + r * Ns;
                    if (last && dst_kind == DST_GLOBAL) {
                        if (qok && e < p.n_out)
                            gdst[t.out_base0 + q * t.out_qstride + (long long)e * p.out_se] =
                                p.post_tw ? post_twiddle(p, v[r], e, t.o) : v[r];
                    } else if (last && dst_kind == DST_TABLE) {
                        // pencils past the end of a ragged tile take the last
                        // valid column (their results are never stored): the
                        // octant fold min(c, L - c) is negative for c > L
                        const int col = t.col0 + min(q, t.nvalid - 1);
                        out_l[lidx<MODE>(q, e, C, L)] = cmul(v[r], table_value<R>(p, e, col, t.o));
                    } else {
                        out_l[lidx<MODE>(q, e, C, L)] = v[r];
                    }
                }
            }
        }
        __syncthreads();
        Ns *= Rr;
    }
}

template <typename R, int MODE, int KIND>
__global__ void __launch_bounds__(256) fft_pass_kernel(PassDesc p) {
    extern __shared__ unsigned char smem_raw[];
    cplx<R>* lds = reinterpret_cast<cplx<R>*>(smem_raw);
    const int CL = p.C * p.L;
    cplx<R>* b0 = lds;
    cplx<R>* b1 = lds + CL;
    cplx<R>* b2 = lds + 2 * CL;
    const Tile t = make_tile<MODE>(p);
    const cplx<R>* gin = reinterpret_cast<const cplx<R>*>(p.in);
    cplx<R>* gout = reinterpret_cast<cplx<R>*>(p.out);
    cplx<R>* gout2 = reinterpret_cast<cplx<R>*>(p.out2);
    if (KIND == KIND_FWD) {
        run_fft<R, MODE, -1>(p, t, SRC_GLOBAL, gin, b0, b1, DST_GLOBAL, gout, nullptr, false, nullptr);
    } else if (KIND == KIND_INV) {
        run_fft<R, MODE, +1>(p, t, SRC_GLOBAL, gin, b0, b1, DST_GLOBAL, gout, nullptr, false, nullptr);
    } else if (KIND == KIND_FUSED) {
        // forward -> Khat -> LDS b2, then inverse from b2 (ping-pong b2 <-> b0)
        run_fft<R, MODE, -1>(p, t, SRC_GLOBAL, gin, b0, b1, DST_TABLE, nullptr, b2, false, nullptr);
        run_fft<R, MODE, +1>(p, t, SRC_LDS, nullptr, b2, b0, DST_GLOBAL, gout, nullptr, false, nullptr);
    } else if (KIND == KIND_FUSED_GRAD) {
        // forward -> Khat -> plain spectrum in b2, i*kappa spectrum in b1
        run_fft<R, MODE, -1>(p, t, SRC_GLOBAL, gin, b0, b1, DST_TABLE, nullptr, b2, false, nullptr);
        // b1 was the ping-pong partner of the forward run; refill it now
        for (int i = threadIdx.x; i < CL; i += blockDim.x) {
            int q, e;
            if (MODE == MODE_COL) {
                q = i % p.C;
                e = i / p.C;
            } else {
                e = i % p.L;
                q = i / p.L;
            }
            b1[i] = times_ikappa(b2[i], axis_index(p, e, t.o), axis_len(p), p.kscale);
            (void)q;
        }
        __syncthreads();
        run_fft<R, MODE, +1>(p, t, SRC_LDS, nullptr, b2, b0, DST_GLOBAL, gout, nullptr, false, nullptr);
        run_fft<R, MODE, +1>(p, t, SRC_LDS, nullptr, b1, b0, DST_GLOBAL, gout2, nullptr, false, nullptr);
    } else if (KIND == KIND_FUSED_DERIV) {
        // forward -> Khat -> b2; i*kappa spectrum in b1; inverse of b1 only
        run_fft<R, MODE, -1>(p, t, SRC_GLOBAL, gin, b0, b1, DST_TABLE, nullptr, b2, false, nullptr);
        for (int i = threadIdx.x; i < CL; i += blockDim.x) {
            const int e = MODE == MODE_COL ? i / p.C : i % p.L;
            b1[i] = times_ikappa(b2[i], axis_index(p, e, t.o), axis_len(p), p.kscale);
        }
        __syncthreads();
        run_fft<R, MODE, +1>(p, t, SRC_LDS, nullptr, b1, b0, DST_GLOBAL, gout, nullptr, false, nullptr);
    } else if (KIND == KIND_INV_GRAD) {
        // plain inverse to out; the loads also stash i*kappa*input in b2,
        // whose inverse goes to out2
        run_fft<R, MODE, +1>(p, t, SRC_GLOBAL, gin, b0, b1, DST_GLOBAL, gout, nullptr, false, b2);
        run_fft<R, MODE, +1>(p, t, SRC_LDS, nullptr, b2, b0, DST_GLOBAL, gout2, nullptr, false, nullptr);
    }
}

// derivative-only inverse: input times i*kappa, then inverse
template <typename R, int MODE>
__global__ void __launch_bounds__(256) fft_inv_deriv_kernel(PassDesc p) {
    extern __shared__ unsigned char smem_raw[];
    cplx<R>* lds = reinterpret_cast<cplx<R>*>(smem_raw);
    const int CL = p.C * p.L;
    const Tile t = make_tile<MODE>(p);
    run_fft<R, MODE, +1>(p, t, SRC_GLOBAL, reinterpret_cast<const cplx<R>*>(p.in), lds, lds + CL, DST_GLOBAL,
                         reinterpret_cast<cplx<R>*>(p.out), nullptr, true, nullptr);
}

int lds_buffers(int kind) {
    return (kind == KIND_FUSED || kind == KIND_FUSED_GRAD || kind == KIND_FUSED_DERIV || kind == KIND_INV_GRAD) ? 3 : 2;
}

template <typename R, int MODE>
hipError_t launch_typed(const PassDesc& p, int kind, bool deriv_only, hipStream_t s) {
    const int nbuf = lds_buffers(kind);
    const size_t lds = (size_t)nbuf * p.C * p.L * sizeof(cplx<R>);
    long long nblocks;
    if (MODE == MODE_COL) {
        nblocks = (long long)p.outer * ((p.inner + p.C - 1) / p.C);
    } else {
        nblocks = (p.outer + p.C - 1) / p.C;
    }
    if (nblocks <= 0) return hipSuccess;
    if (nblocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    int minr = 8;
    for (int i = 0; i < p.nst; ++i) minr = p.radix[i] < minr ? p.radix[i] : minr;
    int nt = (p.C * p.L) / minr;
    nt = nt < 64 ? 64 : (nt > 256 ? 256 : ((nt + 63) / 64) * 64);
    const dim3 grid((unsigned)nblocks), block(nt);
    void (*fn)(PassDesc) = nullptr;
    if (deriv_only) {
        fn = fft_inv_deriv_kernel<R, MODE>;
    } else {
        switch (kind) {
            case KIND_FWD: fn = fft_pass_kernel<R, MODE, KIND_FWD>; break;
            case KIND_INV: fn = fft_pass_kernel<R, MODE, KIND_INV>; break;
            case KIND_FUSED: fn = fft_pass_kernel<R, MODE, KIND_FUSED>; break;
            case KIND_FUSED_GRAD: fn = fft_pass_kernel<R, MODE, KIND_FUSED_GRAD>; break;
            case KIND_FUSED_DERIV: fn = fft_pass_kernel<R, MODE, KIND_FUSED_DERIV>; break;
            case KIND_INV_GRAD: fn = fft_pass_kernel<R, MODE, KIND_INV_GRAD>; break;
            default: return hipErrorInvalidValue;
        }
    }
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(fn, grid, block, lds, s, p);
    return hipGetLastError();
}

}  // namespace

size_t fft_pass_lds_bytes(const PassDesc& p, int kind, bool fp64) {
    return (size_t)lds_buffers(kind) * p.C * p.L * (fp64 ? 16 : 8);
}

int fast_pass_C(int L, int mode, bool fp64);
hipError_t launch_fast_pass(const PassDesc& p, int mode, int kind, bool fp64, hipStream_t s);

// kind values >= 100 select the derivative-only inverse (kind - 100 ignored).
// Steps the plan marked specialised run the length-specialised kernels;
// everything else runs the generic kernel.
hipError_t launch_fft_pass(const PassDesc& p, int mode, int kind, bool fp64, hipStream_t s) {
    if (p.specialised) return launch_fast_pass(p, mode, kind, fp64, s);
    const bool deriv_only = kind >= 100;
    if (deriv_only) kind = KIND_INV;
    if (fp64) {
        return mode == MODE_COL ? launch_typed<double, MODE_COL>(p, kind, deriv_only, s)
                                : launch_typed<double, MODE_ROW>(p, kind, deriv_only, s);
    }
    return mode == MODE_COL ? launch_typed<float, MODE_COL>(p, kind, deriv_only, s)
                            : launch_typed<float, MODE_ROW>(p, kind, deriv_only, s);
}

}  // namespace vg
