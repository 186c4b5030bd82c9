// Length-specialised FFT passes (same contract as fft_pass.hip, faster).
//
// The transform length L, pencils per workgroup C and workgroup size NT are
// compile-time constants, so every index is folded.  Each thread keeps
// E = C L / NT values in registers; a Stockham stage of radix R runs E/R
// butterflies per thread on registers, and consecutive stages exchange data
// through ONE LDS buffer of C L values (store, barrier, load, barrier).
//
// Fusion.  The last forward stage leaves the thread holding exactly the
// spectral values its first inverse butterflies need (the inverse uses the
// forward radix plan reversed), so the Khat multiply (and the i*kappa multiply
// of the gradient kinds) happens in registers between the two transforms with
// no LDS round trip.  Zero-padded inputs (e >= n_in) are never loaded and
// cropped outputs (e >= n_out) are never stored.
//
// Launch geometry.  Column passes give 16 adjacent pencils (128-byte runs for
// complex64) to a workgroup.  Workgroups are dispatched round-robin over the
// 8 XCDs of gfx950; the block index is permuted so that consecutive tiles run
// on the same XCD and share its L2 and TLB.
#pragma once

#include "common.h"
#include "butterfly.h"

namespace vg {

namespace fastfft {

struct RP {
    int n;
    int r[kMaxStages];
};

constexpr RP make_plan(int L) {
    RP p{};
    p.n = 0;
    int x = L, a = 0;
    while (x % 2 == 0) {
        x /= 2;
        ++a;
    }
    while (a >= 3) {
        p.r[p.n++] = 8;
        a -= 3;
    }
    if (a == 2) p.r[p.n++] = 4;
    if (a == 1) p.r[p.n++] = 2;
    const int odd[3] = {3, 5, 7};
    for (int i = 0; i < 3; ++i)
        while (x % odd[i] == 0) {
            x /= odd[i];
            p.r[p.n++] = odd[i];
        }
    return p;
}

constexpr RP reversed(RP p) {
    RP q{};
    q.n = p.n;
    for (int i = 0; i < p.n; ++i) q.r[i] = p.r[p.n - 1 - i];
    return q;
}

constexpr int ns_before(RP p, int s) {
    int v = 1;
    for (int i = 0; i < s; ++i) v *= p.r[i];
    return v;
}

template <int L, int C, int MODE>
struct Lay {
    // LDS slot of element e of pencil q.  Column tiles: pencil index fastest
    // (lanes of a wave touch consecutive slots).  Row tiles: element index
    // fastest, with one padding slot per 16 to break power-of-two strides.
    static constexpr int LP = L + L / 16;
    static constexpr int size = MODE == MODE_COL ? C * L : C * LP;
    __device__ static __forceinline__ int idx(int q, int e) {
        if constexpr (MODE == MODE_COL) return e * C + q;
        else return q * LP + e + (e >> 4);
    }
};

template <int L, int C, int NT, int MODE, int RAD>
__device__ __forceinline__ void bmap(int t, int i, int& q, int& j) {
    constexpr int LR = L / RAD;
    const int b = t + i * NT;
    if constexpr (MODE == MODE_COL) {
        q = b % C;
        j = b / C;
    } else {
        j = b % LR;
        q = b / LR;
    }
}

// Loads and stores at a uniform (scalar) base plus a 32-bit per-lane byte
// offset: the address form global memory instructions take natively, which
// keeps 64-bit address arithmetic off the vector ALU.
template <typename T>
__device__ __forceinline__ T ld_off(const void* base, unsigned off) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off);
}
template <typename T>
__device__ __forceinline__ void st_off(void* base, unsigned off, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off) = v;
}

template <int DIR, typename R>
__device__ __forceinline__ cplx<R> twmul(cplx<R> v, cplx<R> w) {
    return DIR < 0 ? cmul(v, w) : cmulc(v, w);
}

// twiddles and butterflies of stage s of plan P for all of this thread's butterflies
template <typename R, int L, int C, int NT, int MODE, int DIR, RP P, int s>
__device__ __forceinline__ void compute_stage(cplx<R>* v, int t, const cplx<R>* __restrict__ tw) {
    constexpr int RAD = P.r[s];
    constexpr int NS = ns_before(P, s);
    constexpr int E = C * L / NT;
    constexpr int B = E / RAD;
    static_assert(E % RAD == 0, "radix must divide the per-thread element count");
#pragma unroll
    for (int i = 0; i < B; ++i) {
        if constexpr (NS > 1) {
            int q, j;
            bmap<L, C, NT, MODE, RAD>(t, i, q, j);
            const int k = j % NS;
            constexpr int STW = L / (NS * RAD);
#pragma unroll
            for (int r = 1; r < RAD; ++r)
                v[i * RAD + r] = twmul<DIR>(v[i * RAD + r], ld_off<cplx<R>>(tw, (unsigned)(r * k * STW) * sizeof(cplx<R>)));
        }
        dft_fixed<RAD, DIR>(&v[i * RAD]);
    }
}

// outputs of stage s -> LDS, barrier, inputs of stage s+1 <- LDS, barrier
template <typename R, int L, int C, int NT, int MODE, RP P, int s>
__device__ __forceinline__ void exchange(cplx<R>* v, cplx<R>* lds, int t) {
    using LY = Lay<L, C, MODE>;
    constexpr int RAD = P.r[s];
    constexpr int NS = ns_before(P, s);
    constexpr int E = C * L / NT;
#pragma unroll
    for (int i = 0; i < E / RAD; ++i) {
        int q, j;
        bmap<L, C, NT, MODE, RAD>(t, i, q, j);
        const int ob = (j / NS) * NS * RAD + (j % NS);
#pragma unroll
        for (int r = 0; r < RAD; ++r) lds[LY::idx(q, ob + r * NS)] = v[i * RAD + r];
    }
    __syncthreads();
    constexpr int RN = P.r[s + 1];
#pragma unroll
    for (int i = 0; i < E / RN; ++i) {
        int q, j;
        bmap<L, C, NT, MODE, RN>(t, i, q, j);
#pragma unroll
        for (int r = 0; r < RN; ++r) v[i * RN + r] = lds[LY::idx(q, j + r * (L / RN))];
    }
    __syncthreads();
}

template <typename R, int L, int C, int NT, int MODE, int DIR, RP P, int s>
__device__ __forceinline__ void run_from(cplx<R>* v, cplx<R>* lds, int t, const cplx<R>* __restrict__ tw) {
    compute_stage<R, L, C, NT, MODE, DIR, P, s>(v, t, tw);
    if constexpr (s + 1 < P.n) {
        exchange<R, L, C, NT, MODE, P, s>(v, lds, t);
        run_from<R, L, C, NT, MODE, DIR, P, s + 1>(v, lds, t, tw);
    }
}

// ----------------------------------------------------------- tile & I/O --
struct FTile {
    long long in0, out0;    // pencil q = 0
    long long iq, oq;       // pencil stride
    int nvalid;
    int col0;
};

template <int C, int MODE>
__device__ __forceinline__ FTile fast_tile(const PassDesc& p) {
    // XCD-aware permutation: dispatch slot b runs on XCD b % 8; give each XCD a
    // contiguous range of tiles.
    const unsigned nb = gridDim.x;
    unsigned b = blockIdx.x;
    if ((nb & 7u) == 0u) b = (b & 7u) * (nb >> 3) + (b >> 3);
    FTile t;
    if constexpr (MODE == MODE_COL) {
        const int ntile = (p.inner + C - 1) / C;
        const long long o = b / ntile;
        const int c0 = (int)(b % ntile) * C;
        t.in0 = o * p.in_so + c0;
        t.out0 = o * p.out_so + c0;
        t.iq = 1;
        t.oq = 1;
        t.nvalid = min(C, p.inner - c0);
        t.col0 = c0;
    } else {
        const long long o0 = (long long)b * C;
        t.in0 = o0 * p.in_so;
        t.out0 = o0 * p.out_so;
        t.iq = p.in_so;
        t.oq = p.out_so;
        t.nvalid = (int)min((long long)C, (long long)p.outer - o0);
        t.col0 = 0;
    }
    return t;
}

__device__ __forceinline__ int sfreq(int e, int L) {
    const int h = L >> 1;
    return e < h ? e : (e == h ? 0 : e - L);
}

template <typename R>
__device__ __forceinline__ cplx<R> ikap(cplx<R> v, int e, int L, R ks) {
    const R kap = ks * (R)sfreq(e, L);
    return mk(-kap * v.y, kap * v.x);
}

// global -> registers for stage 0 of plan P (entries e >= NIN are zero).
// Element e = j + r L/R of pencil q: the part r (L/R) se is uniform and goes
// into the scalar base; the lane offset (q iq + j se) * size stays below 2^32
// (checked by the host dispatcher).  Pencils past the end of a ragged tile
// read the tile's last pencil (in bounds; their results are never stored).
template <typename R, int L, int C, int NT, int MODE, RP P, int NIN>
__device__ __forceinline__ void load_global(cplx<R>* v, const cplx<R>* __restrict__ g, const FTile& tl,
                                            long long se, int t) {
    constexpr int RAD = P.r[0];
    constexpr int E = C * L / NT;
    constexpr int LR = L / RAD;
    unsigned off[E / RAD];
    int jj[E / RAD];
#pragma unroll
    for (int i = 0; i < E / RAD; ++i) {
        int q, j;
        bmap<L, C, NT, MODE, RAD>(t, i, q, j);
        q = min(q, tl.nvalid - 1);
        off[i] = (unsigned)((long long)q * tl.iq + (long long)j * se) * (unsigned)sizeof(cplx<R>);
        jj[i] = j;
    }
#pragma unroll
    for (int r = 0; r < RAD; ++r) {
        const cplx<R>* gb = g + tl.in0 + (long long)(r * LR) * se;
#pragma unroll
        for (int i = 0; i < E / RAD; ++i) {
            cplx<R> x = mk(R(0), R(0));
            if ((r + 1) * LR <= NIN || (r * LR < NIN && jj[i] + r * LR < NIN)) x = ld_off<cplx<R>>(gb, off[i]);
            v[i * RAD + r] = x;
        }
    }
}

// registers (outputs of the last stage of plan P) -> global, e < NOUT only.
// Outputs never stored are dead, so their arithmetic is dropped by the compiler.
template <typename R, int L, int C, int NT, int MODE, RP P, int NOUT, bool FULL>
__device__ __forceinline__ void store_global_t(const cplx<R>* v, cplx<R>* __restrict__ g, const FTile& tl,
                                               long long se, int t) {
    constexpr int RAD = P.r[P.n - 1];
    constexpr int E = C * L / NT;
    constexpr int LR = L / RAD;
    unsigned off[E / RAD];
    int jj[E / RAD];
    bool ok[E / RAD];
#pragma unroll
    for (int i = 0; i < E / RAD; ++i) {
        int q, j;
        bmap<L, C, NT, MODE, RAD>(t, i, q, j);
        ok[i] = FULL || q < tl.nvalid;
        off[i] = (unsigned)((long long)q * tl.oq + (long long)j * se) * (unsigned)sizeof(cplx<R>);
        jj[i] = j;
    }
#pragma unroll
    for (int r = 0; r < RAD; ++r) {
        if (r * LR < NOUT) {
            cplx<R>* gb = g + tl.out0 + (long long)(r * LR) * se;
#pragma unroll
            for (int i = 0; i < E / RAD; ++i)
                if (ok[i] && ((r + 1) * LR <= NOUT || jj[i] + r * LR < NOUT)) st_off(gb, off[i], v[i * RAD + r]);
        }
    }
}

template <typename R, int L, int C, int NT, int MODE, RP P, int NOUT>
__device__ __forceinline__ void store_global(const cplx<R>* v, cplx<R>* __restrict__ g, const FTile& tl,
                                             long long se, int t) {
    if (tl.nvalid == C) store_global_t<R, L, C, NT, MODE, P, NOUT, true>(v, g, tl, se, t);
    else store_global_t<R, L, C, NT, MODE, P, NOUT, false>(v, g, tl, se, t);
}

// Khat octant values for the thread's spectral positions (last-stage outputs
// of plan P), loaded before the forward transform so that their latency hides
// behind it; d == 3: column c = k2 * L + k3, d == 2: column c = k2.
template <typename R, int L, int C, int NT, int MODE, RP P, int D, bool CPLX>
__device__ __forceinline__ void table_fetch(cplx<R>* kt, const void* __restrict__ table, int tabN, int col0,
                                            int nvalid, int t) {
    constexpr int RAD = P.r[P.n - 1];
    constexpr int E = C * L / NT;
    const int N1 = tabN + 1;
    const unsigned plane = (D == 3) ? (unsigned)(N1 * N1) : (unsigned)N1;
#pragma unroll
    for (int i = 0; i < E / RAD; ++i) {
        int q, j;
        bmap<L, C, NT, MODE, RAD>(t, i, q, j);
        const int col = min(col0 + q, col0 + nvalid - 1);
        unsigned rowoff;
        if constexpr (D == 3) {
            const int k2 = col / L, k3 = col % L;
            rowoff = (unsigned)(min(k2, L - k2) * N1 + min(k3, L - k3));
        } else {
            rowoff = (unsigned)min(col, L - col);
        }
        const unsigned jp = (unsigned)j * plane;
#pragma unroll
        for (int r = 0; r < RAD; ++r) {
            // e = j + r L/R with 0 <= j < L/R: the octant fold min(e, L - e) is
            // e on blocks below L/2 and L - e on blocks at or above it.
            constexpr int LR = L / RAD;
            const int e = j + r * LR;
            unsigned flat;
            if ((r + 1) * LR <= L / 2) flat = (unsigned)(r * LR) * plane + jp + rowoff;
            else if (r * LR >= L / 2) flat = (unsigned)(L - r * LR) * plane - jp + rowoff;
            else flat = (unsigned)min(e, L - e) * plane + rowoff;
            if constexpr (CPLX) {
                kt[i * RAD + r] = ld_off<cplx<R>>(table, flat * (unsigned)sizeof(cplx<R>));
            } else {
                kt[i * RAD + r] = mk(ld_off<R>(table, flat * (unsigned)sizeof(R)), R(0));
            }
        }
    }
}

template <typename R, int E, bool CPLX>
__device__ __forceinline__ void table_apply(cplx<R>* v, const cplx<R>* kt) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if constexpr (CPLX) v[e] = cmul(v[e], kt[e]);
        else v[e] = mk(v[e].x * kt[e].x, v[e].y * kt[e].x);
    }
}

// v2 = i*kappa(e) * v at the stage-0 input positions (plan P) or last-stage
// output positions (LAST) -- both are e = j + r L/R.
template <typename R, int L, int C, int NT, int MODE, int RAD>
__device__ __forceinline__ void deriv_copy(const cplx<R>* v, cplx<R>* v2, R ks, int t) {
    constexpr int E = C * L / NT;
#pragma unroll
    for (int i = 0; i < E / RAD; ++i) {
        int q, j;
        bmap<L, C, NT, MODE, RAD>(t, i, q, j);
#pragma unroll
        for (int r = 0; r < RAD; ++r) v2[i * RAD + r] = ikap(v[i * RAD + r], j + r * (L / RAD), L, ks);
    }
}

enum FastKind : int { FK_FWD = 0, FK_INV = 1, FK_FUSED = 2, FK_FUSED_GRAD = 3, FK_INV_GRAD = 4, FK_INV_DERIV = 5 };

template <typename R, int L, int C, int NT, int MODE, int FK, int D, bool CPLX>
__global__ void __launch_bounds__(NT) fast_kernel(PassDesc p) {
    constexpr RP F = make_plan(L);
    constexpr RP I = reversed(F);
    constexpr int E = C * L / NT;
    using LY = Lay<L, C, MODE>;
    __shared__ cplx<R> lds[LY::size];
    const int t = threadIdx.x;
    const FTile tl = fast_tile<C, MODE>(p);
    const cplx<R>* __restrict__ tw = reinterpret_cast<const cplx<R>*>(p.tw);
    const cplx<R>* __restrict__ gin = reinterpret_cast<const cplx<R>*>(p.in);
    cplx<R>* __restrict__ gout = reinterpret_cast<cplx<R>*>(p.out);
    cplx<R>* __restrict__ gout2 = reinterpret_cast<cplx<R>*>(p.out2);
    const R ks = (R)p.kscale;
    cplx<R> v[E];
    if constexpr (FK == FK_FWD) {
        load_global<R, L, C, NT, MODE, F, L / 2>(v, gin, tl, p.in_se, t);
        run_from<R, L, C, NT, MODE, -1, F, 0>(v, lds, t, tw);
        store_global<R, L, C, NT, MODE, F, L>(v, gout, tl, p.out_se, t);
    } else if constexpr (FK == FK_INV || FK == FK_INV_DERIV) {
        load_global<R, L, C, NT, MODE, I, L>(v, gin, tl, p.in_se, t);
        if constexpr (FK == FK_INV_DERIV) {
            cplx<R> w[E];
            deriv_copy<R, L, C, NT, MODE, I.r[0]>(v, w, ks, t);
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = w[e];
        }
        run_from<R, L, C, NT, MODE, +1, I, 0>(v, lds, t, tw);
        store_global<R, L, C, NT, MODE, I, L / 2>(v, gout, tl, p.out_se, t);
    } else if constexpr (FK == FK_INV_GRAD) {
        load_global<R, L, C, NT, MODE, I, L>(v, gin, tl, p.in_se, t);
        cplx<R> w[E];
        deriv_copy<R, L, C, NT, MODE, I.r[0]>(v, w, ks, t);
        run_from<R, L, C, NT, MODE, +1, I, 0>(v, lds, t, tw);
        store_global<R, L, C, NT, MODE, I, L / 2>(v, gout, tl, p.out_se, t);
        __syncthreads();
        run_from<R, L, C, NT, MODE, +1, I, 0>(w, lds, t, tw);
        store_global<R, L, C, NT, MODE, I, L / 2>(w, gout2, tl, p.out_se, t);
    } else {
        // FK_FUSED, FK_FUSED_GRAD
        cplx<R> kt[E];
        load_global<R, L, C, NT, MODE, F, L / 2>(v, gin, tl, p.in_se, t);
        table_fetch<R, L, C, NT, MODE, F, D, CPLX>(kt, p.table, p.tabN, tl.col0, tl.nvalid, t);
        run_from<R, L, C, NT, MODE, -1, F, 0>(v, lds, t, tw);
        table_apply<R, E, CPLX>(v, kt);
        if constexpr (FK == FK_FUSED) {
            run_from<R, L, C, NT, MODE, +1, I, 0>(v, lds, t, tw);
            store_global<R, L, C, NT, MODE, I, L / 2>(v, gout, tl, p.out_se, t);
        } else {
            cplx<R> w[E];
            deriv_copy<R, L, C, NT, MODE, F.r[F.n - 1]>(v, w, ks, t);
            run_from<R, L, C, NT, MODE, +1, I, 0>(v, lds, t, tw);
            store_global<R, L, C, NT, MODE, I, L / 2>(v, gout, tl, p.out_se, t);
            __syncthreads();
            run_from<R, L, C, NT, MODE, +1, I, 0>(w, lds, t, tw);
            store_global<R, L, C, NT, MODE, I, L / 2>(w, gout2, tl, p.out_se, t);
        }
    }
}

// --------------------------------------------------------------- dispatch --
template <typename R, int L, int C, int NT, int MODE>
hipError_t launch_shape(const PassDesc& p, int kind, hipStream_t s) {
    long long nblocks = MODE == MODE_COL ? (long long)p.outer * ((p.inner + C - 1) / C) : (p.outer + C - 1) / C;
    if (nblocks <= 0) return hipSuccess;
    if (nblocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)nblocks), block(NT);
    const bool fused = kind == KIND_FUSED || kind == KIND_FUSED_GRAD;
    if (fused && MODE == MODE_COL) {
        const bool g = kind == KIND_FUSED_GRAD;
#define VG_FUSED_LAUNCH(DD, CX)                                                                          \
    if (g) {                                                                                             \
        hipLaunchKernelGGL((fast_kernel<R, L, C, NT, MODE, FK_FUSED_GRAD, DD, CX>), grid, block, 0, s, p); \
    } else {                                                                                             \
        hipLaunchKernelGGL((fast_kernel<R, L, C, NT, MODE, FK_FUSED, DD, CX>), grid, block, 0, s, p);      \
    }
        if (p.d == 3 && p.table_complex) {
            VG_FUSED_LAUNCH(3, true)
        } else if (p.d == 3) {
            VG_FUSED_LAUNCH(3, false)
        } else if (p.table_complex) {
            VG_FUSED_LAUNCH(2, true)
        } else {
            VG_FUSED_LAUNCH(2, false)
        }
#undef VG_FUSED_LAUNCH
        return hipGetLastError();
    }
    switch (kind) {
        case KIND_FWD: hipLaunchKernelGGL((fast_kernel<R, L, C, NT, MODE, FK_FWD, 3, false>), grid, block, 0, s, p); break;
        case KIND_INV: hipLaunchKernelGGL((fast_kernel<R, L, C, NT, MODE, FK_INV, 3, false>), grid, block, 0, s, p); break;
        case KIND_INV_GRAD:
            hipLaunchKernelGGL((fast_kernel<R, L, C, NT, MODE, FK_INV_GRAD, 3, false>), grid, block, 0, s, p);
            break;
        case 100 + KIND_INV:
            hipLaunchKernelGGL((fast_kernel<R, L, C, NT, MODE, FK_INV_DERIV, 3, false>), grid, block, 0, s, p);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Launch shape per (length, mode, element size): C pencils per workgroup, E
// values per thread (a multiple of every radix of the plan), NT = C L / E
// threads.  LDS (C pencils, row tiles padded) stays within 64 KiB; tiny
// lengths take more pencils so a workgroup has at least one full wave.
struct Shape {
    int C, E, NT;
};

constexpr int gcd_i(int a, int b) { return b == 0 ? a : gcd_i(b, a % b); }

constexpr Shape shape_for(int L, int mode, int esize) {
    const RP p = make_plan(L);
    int lc = 1;
    for (int i = 0; i < p.n; ++i) lc = lc / gcd_i(lc, p.r[i]) * p.r[i];
    const int target = esize == 16 ? 16 : 32;
    const int E = lc >= target ? lc : (target / lc) * lc;
    const int LP = mode == MODE_COL ? L : L + L / 16;
    int C = mode == MODE_COL ? 16 : 8;
    while (C > 1 && C * LP * esize > 65536) C /= 2;
    while (C * L / E < 64 && C < 64 && 2 * C * LP * esize <= 65536) C *= 2;
    return Shape{C, E, C * L / E};
}

template <typename R, int L, int MODE>
hipError_t launch_len_mode(const PassDesc& p, int kind, hipStream_t s) {
    constexpr Shape S = shape_for(L, MODE, (int)sizeof(cplx<R>));
    static_assert(S.C * L % S.E == 0 && S.NT >= 64 && S.NT <= 1024, "bad launch shape");
    if (p.C != S.C) return hipErrorInvalidValue;
    return launch_shape<R, L, S.C, S.NT, MODE>(p, kind, s);
}

template <typename R, int L>
hipError_t launch_len(const PassDesc& p, int mode, int kind, hipStream_t s) {
    return mode == MODE_COL ? launch_len_mode<R, L, MODE_COL>(p, kind, s) : launch_len_mode<R, L, MODE_ROW>(p, kind, s);
}

template <typename R, int L>
int shape_C(int mode) {
    return mode == MODE_COL ? shape_for(L, MODE_COL, (int)sizeof(cplx<R>)).C
                            : shape_for(L, MODE_ROW, (int)sizeof(cplx<R>)).C;
}

}  // namespace fastfft

// One translation unit per length instantiates these through
// VG_FAST_INSTANTIATE(L); fft_fast.hip dispatches on the length.
#define VG_FAST_INSTANTIATE(LL)                                                                         \
    int fast_C_##LL(int mode, bool fp64) {                                                              \
        return fp64 ? fastfft::shape_C<double, LL>(mode) : fastfft::shape_C<float, LL>(mode);           \
    }                                                                                                   \
    hipError_t launch_fast_##LL(const PassDesc& p, int mode, int kind, bool fp64, hipStream_t s) {      \
        return fp64 ? fastfft::launch_len<double, LL>(p, mode, kind, s)                                 \
                    : fastfft::launch_len<float, LL>(p, mode, kind, s);                                 \
    }

}  // namespace vg
