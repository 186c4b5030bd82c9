// Length-specialised FFT passes (same contract as fft_pass.hip, faster).
//
// The transform length L, pencils per workgroup C and workgroup size NT are
// compile-time constants, so every index is folded.  Each thread keeps
// E = C L / NT values in registers; a Stockham stage of radix R runs E/R
// butterflies per thread on registers, and consecutive stages exchange data
// through ONE LDS buffer of C L values (store, barrier, load, barrier).
// Complex64 power-of-two lengths use radices up to 32 (512 = 32 x 16), so a
// transform needs one LDS exchange instead of two.
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
// on the same XCD and share its L2 and TLB (and, in the fused passes, so that
// tiles reading the same table entries run next to each other).
//
// Lengths: powers of two up to 1024 (rows and columns) and 8192 (rows), plus
// the mixed-radix 96, 100, 192, 200, 300, 400, 500 and, for rows, 3200, 6400,
// 12800 (one translation unit per length, fft_fast_<L>.hip).
#pragma once

#include <type_traits>

#include "common.h"
#include "butterfly.h"

namespace vg {

namespace fastfft {

struct RP {
    int n;
    int r[kMaxStages];
};

// Radix plan of a specialised length.  Power-of-two lengths take as few
// stages as radices up to MAXR allow, with the bits spread evenly (512 =
// 32 x 16 for complex64); lengths with factors 3, 5, 7 use one stage per odd
// factor and power-of-two radices up to 8.
constexpr RP plan_bits(int L, int mb) {
    RP p{};
    p.n = 0;
    int x = L, a = 0;
    while (x % 2 == 0) {
        x /= 2;
        ++a;
    }
    const int S = (a + mb - 1) / mb;
    for (int i = 0; i < S; ++i) {
        const int bits = a / (S - i) + ((a % (S - i)) ? 1 : 0);
        p.r[p.n++] = 1 << bits;
        a -= bits;
    }
    const int odd[3] = {3, 5, 7};
    for (int i = 0; i < 3; ++i)
        while (x % odd[i] == 0) {
            x /= odd[i];
            p.r[p.n++] = odd[i];
        }
    return p;
}

// least common multiple of a plan's radices: every thread holds a multiple of
// it, one whole butterfly of each stage at a time
constexpr int plan_lcm(const RP& p) {
    int lc = 1;
    for (int i = 0; i < p.n; ++i) {
        int a = lc, b = p.r[i];
        while (b != 0) {
            const int t = a % b;
            a = b;
            b = t;
        }
        lc = lc / a * p.r[i];
    }
    return lc;
}

// Mixed lengths up to 512 (the ones with column passes) shrink their
// power-of-two radices until at most 32 values per thread are needed: 200 =
// 4 x 2 x 5 x 5 instead of 8 x 5 x 5 (40 values), 300 = 2 x 2 x 3 x 5 x 5
// instead of 4 x 3 x 5 x 5 (60 values, 256 VGPRs and one wave per SIMD in
// the fused pass).  The extra exchange costs less than the occupancy gained:
// 3D N = 150 apply 0.430 -> 0.304 ms, N = 100 0.104 -> 0.087 ms.
constexpr RP make_plan(int L, int maxr = 8) {
    int x = L;
    while (x % 2 == 0) x /= 2;
    if (x == 1) return plan_bits(L, maxr >= 32 ? 5 : (maxr >= 16 ? 4 : 3));
    int mb = 3;
    if (L <= 512)
        while (mb > 1 && plan_lcm(plan_bits(L, mb)) > 32) --mb;
    return plan_bits(L, mb);
}

// largest radix used for a precision: complex64 threads hold 32 values
template <typename R>
constexpr int kMaxRad = sizeof(R) == 4 ? 32 : 16;

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

template <int L, int C, int MODE, int ES, int LIM = 65536>
struct Lay {
    // LDS slot of element e of pencil q.  Column tiles: pencil index fastest
    // (lanes of a wave touch consecutive slots).  Row tiles: element index
    // fastest, with one padding slot per 16 (when it fits in LIM bytes) to
    // break power-of-two strides.
    static constexpr bool PAD = MODE == MODE_ROW && C * (L + L / 16) * ES <= LIM;
    static constexpr int LP = PAD ? L + L / 16 : L;
    static constexpr int size = MODE == MODE_COL ? C * L : C * LP;
    __device__ static __forceinline__ int idx(int q, int e) {
        if constexpr (MODE == MODE_COL) return e * C + q;
        else if constexpr (PAD) return q * LP + e + (e >> 4);
        else return q * LP + e;
    }
};

// Column tiles of two-stage plans in the plain fused kernels (CPAD): C
// padding slots after every block of RAD0 = P.r[0] elements, slot
// e C + q + (e / RAD0) C.  The first-stage writes (element j RAD0 + r of
// lane j) then fall in distinct banks.  The block index is j on write and r
// on read (element j + r RAD0 with j < RAD0), so it is added as such: per
// lane or compile-time.  Measured on the fused pass:
// 3D N = 256 -1.6%, N = 512 -0.6%; the gradient kinds of length 1024 were
// slower with it (fused derivative 3.29 -> 3.79 ms), the unfused column
// passes unchanged, so only the plain fused kind uses it.
template <int L, int C, int MODE, RP P, bool CPAD>
struct ColPad {
    static constexpr bool on = CPAD && MODE == MODE_COL && P.n == 2;
    // pad slots before block b
    __host__ __device__ static constexpr int add(int b) { return on ? b * C : 0; }
};
// slots a two-stage column tile needs, padding for either plan's first radix
template <int L, int C, RP F>
constexpr int col_pad_slots() {
    if (F.n != 2) return 0;
    const int r = F.r[0] < F.r[1] ? F.r[0] : F.r[1];
    return C * (L / r);
}

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

// Streaming (non-temporal) access to the pencil data: every element is read
// once and written once per pass, so these loads and stores are marked
// non-temporal and leave the caches to the reused data (twiddles, the Khat
// table).  Loads are streaming in the row passes and in column passes whose
// tile rows cover whole 128-byte lines (C complex values >= 128 bytes, and
// pitches that keep them line-aligned: PassDesc::stream, set by the host);
// otherwise the neighbouring tile reads the other part of each line, which
// an ordinary load leaves in L2.  Stores are streaming in those column
// passes only -- the row passes' outputs are read next (the first column
// pass, or the caller) and stay cache-resident with ordinary stores.
// Measured: 3D N = 256 apply (C = 16 complex64 columns) 0.757 -> 0.696 ms;
// 3D N = 512 apply (C = 8) 8.8 ms streaming vs 7.3 ms ordinary.
template <typename R, int C, int MODE>
constexpr bool streaming_loads() {
    return MODE == MODE_ROW || C * (int)sizeof(cplx<R>) >= 128;
}
template <typename R, int C, int MODE>
constexpr bool streaming_stores() {
    return MODE == MODE_COL && C * (int)sizeof(cplx<R>) >= 128;
}
template <typename R>
__device__ __forceinline__ cplx<R> ld_stream(const void* base, unsigned off) {
    typedef R v2 __attribute__((ext_vector_type(2)));
    const v2 x = __builtin_nontemporal_load(reinterpret_cast<const v2*>(reinterpret_cast<const char*>(base) + off));
    return mk(x.x, x.y);
}
template <typename R>
__device__ __forceinline__ void st_stream(void* base, unsigned off, cplx<R> c) {
    typedef R v2 __attribute__((ext_vector_type(2)));
    v2 x;
    x.x = c.x;
    x.y = c.y;
    __builtin_nontemporal_store(x, reinterpret_cast<v2*>(reinterpret_cast<char*>(base) + off));
}

// A value known to be the same in every lane, passed through readfirstlane:
// the compiler keeps it in a scalar register and cannot factor it into
// per-element vector multiplies.
__device__ __forceinline__ unsigned uniform_u32(unsigned v) { return __builtin_amdgcn_readfirstlane(v); }



template <int DIR, typename R>
__device__ __forceinline__ cplx<R> twmul(cplx<R> v, cplx<R> w) {
    return DIR < 0 ? cmul(v, w) : cmulc(v, w);
}

// Stage twiddles of lengths whose table (L entries) is too large for the
// workgroup's LDS copy: two small tables in LDS, tw[0, 64) = W^i and
// tw[64 + i] = W^(64 i), and W^m = W^(64 (m / 64)) W^(m % 64) (one more
// complex product, about one more rounding; the global table had cost the
// 2D N = 4096 rows of length 8192 a third of their time).
template <typename R, int L>
constexpr bool tw_split() {
    return L * (int)sizeof(cplx<R>) > 8192 && L % 64 == 0 && make_plan(L, kMaxRad<R>).n >= 2;
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
            for (int r = 1; r < RAD; ++r) {
                const unsigned m = (unsigned)(r * k * STW);
                cplx<R> w;
                if constexpr (tw_split<R, L>()) w = cmul(tw[64 + (m >> 6)], tw[m & 63u]);
                else w = ld_off<cplx<R>>(tw, m * (unsigned)sizeof(cplx<R>));
                v[i * RAD + r] = twmul<DIR>(v[i * RAD + r], w);
            }
        }
        dft_fixed<RAD, DIR>(&v[i * RAD]);
    }
}

// outputs of stage s -> LDS, barrier, inputs of stage s+1 <- LDS, barrier.
// SPLIT: real parts first, then imaginary parts, through half the LDS.
// Row pencils of the plain (complex) exchange stay padded up to 80 KiB of
// LDS: a single 8192-point complex64 row (68 KiB padded) still leaves room
// for two workgroups per CU, and the padding removes most of its bank
// conflicts (2D N = 4096 forward rows 0.122 -> 0.115 ms).
constexpr int kPadLimit = 81920;

template <typename R, int L, int C, int NT, int MODE, RP P, int s, bool SPLIT, bool CPAD = false>
__device__ __forceinline__ void exchange(cplx<R>* v, cplx<R>* lds, int t) {
    using LY = Lay<L, C, MODE, (int)sizeof(cplx<R>), SPLIT ? 65536 : kPadLimit>;
    using CP = ColPad<L, C, MODE, P, CPAD>;
    constexpr int RAD = P.r[s];
    constexpr int NS = ns_before(P, s);
    constexpr int E = C * L / NT;
    constexpr int RN = P.r[s + 1];
    static_assert(!CP::on || s == 0, "the padded layout covers the one exchange of a two-stage plan");
    // Column slots are linear in the element (e C + q, plus the pad), so the
    // writes of lane (q, j) sit at a lane base plus r NS C and the reads at a
    // lane base plus r BS: immediate offsets, no per-element index
    // arithmetic.  Row tiles keep LY::idx (padded every 16 elements).
    constexpr int BS = (L / RN) * C + CP::add(1);
    auto wslot = [&](int q, int j, int ob, int r) -> int {
        if constexpr (MODE == MODE_COL) return (ob * C + q + CP::add(j)) + r * NS * C;
        else return LY::idx(q, ob + r * NS);
    };
    auto rslot = [&](int q, int j, int r) -> int {
        if constexpr (MODE == MODE_COL) return (j * C + q) + r * BS;
        else return LY::idx(q, j + r * (L / RN));
    };
    if constexpr (SPLIT) {
        R* lr = reinterpret_cast<R*>(lds);
#pragma unroll
        for (int part = 0; part < 2; ++part) {
#pragma unroll
            for (int i = 0; i < E / RAD; ++i) {
                int q, j;
                bmap<L, C, NT, MODE, RAD>(t, i, q, j);
                const int ob = (j / NS) * NS * RAD + (j % NS);
#pragma unroll
                for (int r = 0; r < RAD; ++r) lr[wslot(q, j, ob, r)] = part ? v[i * RAD + r].y : v[i * RAD + r].x;
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < E / RN; ++i) {
                int q, j;
                bmap<L, C, NT, MODE, RN>(t, i, q, j);
#pragma unroll
                for (int r = 0; r < RN; ++r) {
                    const R x = lr[rslot(q, j, r)];
                    if (part) v[i * RN + r].y = x;
                    else v[i * RN + r].x = x;
                }
            }
            __syncthreads();
        }
    } else {
#pragma unroll
        for (int i = 0; i < E / RAD; ++i) {
            int q, j;
            bmap<L, C, NT, MODE, RAD>(t, i, q, j);
            const int ob = (j / NS) * NS * RAD + (j % NS);
#pragma unroll
            for (int r = 0; r < RAD; ++r) lds[wslot(q, j, ob, r)] = v[i * RAD + r];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < E / RN; ++i) {
            int q, j;
            bmap<L, C, NT, MODE, RN>(t, i, q, j);
#pragma unroll
            for (int r = 0; r < RN; ++r) v[i * RN + r] = lds[rslot(q, j, r)];
        }
        __syncthreads();
    }
}

template <typename R, int L, int C, int NT, int MODE, int DIR, RP P, int s, bool SPLIT = false, bool CPAD = false>
__device__ __forceinline__ void run_from(cplx<R>* v, cplx<R>* lds, int t, const cplx<R>* __restrict__ tw) {
    compute_stage<R, L, C, NT, MODE, DIR, P, s>(v, t, tw);
    if constexpr (s + 1 < P.n) {
        exchange<R, L, C, NT, MODE, P, s, SPLIT, CPAD>(v, lds, t);
        run_from<R, L, C, NT, MODE, DIR, P, s + 1, SPLIT, CPAD>(v, lds, t, tw);
    }
}

// ----------------------------------------------------------- tile & I/O --
struct FTile {
    long long in0, out0;    // pencil q = 0
    long long iq, oq;       // pencil stride
    int nvalid;
    int col0;
    int o;                  // outer index (column tiles)
    int stream;             // streaming access allowed (PassDesc::stream: 1 loads, 2 stores)
};

// XCD-aware order for one-tile-per-workgroup launches: dispatch slot b runs
// on XCD b % 8; give each XCD a contiguous range of tiles.
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned nb) {
    return ((nb & 7u) == 0u) ? (b & 7u) * (nb >> 3) + (b >> 3) : b;
}

template <int C, int MODE>
__device__ __forceinline__ FTile fast_tile(const PassDesc& p, unsigned b) {
    FTile t;
    t.stream = p.stream;
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
        t.o = (int)o;
    } else {
        const long long o0 = (long long)b * C;
        t.in0 = o0 * p.in_so;
        t.out0 = o0 * p.out_so;
        t.iq = p.in_so;
        t.oq = p.out_so;
        t.nvalid = (int)min((long long)C, (long long)p.outer - o0);
        t.col0 = 0;
        t.o = 0;
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
// Only blocks r with r L/R < NIN are loaded (NR of them); expand() places the
// loaded values and the zeros into stage order.
template <typename R, int L, int C, int NT, RP P, int NIN>
struct LoadSet {
    static constexpr int RAD = P.r[0];
    static constexpr int E = C * L / NT;
    static constexpr int LR = L / RAD;
    static constexpr int NR = ((NIN + LR - 1) / LR) < RAD ? (NIN + LR - 1) / LR : RAD;
    static constexpr int NV = (E / RAD) * NR;
};

template <typename R, int L, int C, int NT, int MODE, RP P, int NIN>
__device__ __forceinline__ void issue_loads(cplx<R>* vn, const cplx<R>* __restrict__ g, const FTile& tl,
                                            long long se, int t) {
    using LS = LoadSet<R, L, C, NT, P, NIN>;
    constexpr int RAD = LS::RAD, LR = LS::LR, NR = LS::NR, NB = LS::E / RAD;
    unsigned off[NB];
    int jj[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        int q, j;
        bmap<L, C, NT, MODE, RAD>(t, i, q, j);
        q = min(q, tl.nvalid - 1);
        off[i] = (unsigned)((long long)q * tl.iq + (long long)j * se) * (unsigned)sizeof(cplx<R>);
        jj[i] = j;
    }
    auto body = [&](auto stream) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const cplx<R>* gb = g + tl.in0 + (long long)(r * LR) * se;
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                cplx<R> x = mk(R(0), R(0));
                if ((r + 1) * LR <= NIN || jj[i] + r * LR < NIN) {
                    if constexpr (decltype(stream)::value) x = ld_stream<R>(gb, off[i]);
                    else x = ld_off<cplx<R>>(gb, off[i]);
                }
                vn[i * NR + r] = x;
            }
        }
    };
    if (streaming_loads<R, C, MODE>() && (tl.stream & 1)) body(std::true_type{});
    else body(std::false_type{});
}

template <typename R, int L, int C, int NT, RP P, int NIN>
__device__ __forceinline__ void expand(cplx<R>* v, const cplx<R>* vn) {
    using LS = LoadSet<R, L, C, NT, P, NIN>;
    constexpr int RAD = LS::RAD, NR = LS::NR, NB = LS::E / RAD;
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int r = 0; r < RAD; ++r) v[i * RAD + r] = r < NR ? vn[i * NR + r] : mk(R(0), R(0));
}

// registers (outputs of the last stage of plan P) -> global, e < NOUT only.
// Outputs never stored are dead, so their arithmetic is dropped by the compiler.
// PT (four-step passes): multiply output e by W_{L_big}^{o e} (1) or its
// conjugate (2) from the table tw_big, o the tile's outer index.
template <typename R, int L, int C, int NT, int MODE, RP P, int NOUT, bool FULL, int PT>
__device__ __forceinline__ void store_global_t(const cplx<R>* v, cplx<R>* __restrict__ g, const FTile& tl,
                                               long long se, int t, const void* __restrict__ twb) {
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
    auto body = [&](auto stream) {
#pragma unroll
        for (int r = 0; r < RAD; ++r) {
            if (r * LR < NOUT) {
                cplx<R>* gb = g + tl.out0 + (long long)(r * LR) * se;
#pragma unroll
                for (int i = 0; i < E / RAD; ++i) {
                    cplx<R> x = v[i * RAD + r];
                    if constexpr (PT != 0) {
                        const cplx<R> w =
                            ld_off<cplx<R>>(twb, (unsigned)(tl.o * (jj[i] + r * LR)) * (unsigned)sizeof(cplx<R>));
                        x = PT == 1 ? cmul(x, w) : cmulc(x, w);
                    }
                    if (ok[i] && ((r + 1) * LR <= NOUT || jj[i] + r * LR < NOUT)) {
                        if constexpr (decltype(stream)::value) st_stream<R>(gb, off[i], x);
                        else st_off(gb, off[i], x);
                    }
                }
            }
        }
    };
    if (streaming_stores<R, C, MODE>() && (tl.stream & 2)) body(std::true_type{});
    else body(std::false_type{});
}

template <typename R, int L, int C, int NT, int MODE, RP P, int NOUT, int PT = 0>
__device__ __forceinline__ void store_global(const cplx<R>* v, cplx<R>* __restrict__ g, const FTile& tl,
                                             long long se, int t, const void* twb = nullptr) {
    if (tl.nvalid == C) store_global_t<R, L, C, NT, MODE, P, NOUT, true, PT>(v, g, tl, se, t, twb);
    else store_global_t<R, L, C, NT, MODE, P, NOUT, false, PT>(v, g, tl, se, t, twb);
}

// Khat octant values for the thread's spectral positions (last-stage outputs
// of plan P), loaded before the forward transform so that their latency hides
// behind it; d == 3: column c = k2 * L + k3, d == 2: column c = k2.
// HALF: real-data plans keep the half spectrum k3 in [0, N] of the last axis;
// the column is then c = k2 (N + 1) + k3 (3D) or c = k2 (2D), k3 / k2 unfolded.
// FULL: the table holds every spectral index (convection kernel): flat =
// e L^(d-1) + c.
template <typename R, int L, int C, int NT, int MODE, RP P, int D, bool CPLX, bool HALF = false, bool FULL = false>
__device__ __forceinline__ void table_fetch(cplx<R>* kt, const void* __restrict__ table, int tabN, int tp,
                                            int col0, int nvalid, int t) {
    constexpr int RAD = P.r[P.n - 1];
    constexpr int E = C * L / NT;
    if constexpr (FULL) {
        constexpr unsigned plane = D == 3 ? (unsigned)L * (unsigned)L : (unsigned)L;
#pragma unroll
        for (int i = 0; i < E / RAD; ++i) {
            int q, j;
            bmap<L, C, NT, MODE, RAD>(t, i, q, j);
            const unsigned col = (unsigned)min(col0 + q, col0 + nvalid - 1);
#pragma unroll
            for (int r = 0; r < RAD; ++r) {
                const unsigned flat = (unsigned)(j + r * (L / RAD)) * plane + col;
                kt[i * RAD + r] = ld_off<cplx<R>>(table, flat * (unsigned)sizeof(cplx<R>));
            }
        }
        return;
    }
    const int N1 = tabN + 1;
    // block strides as opaque scalars: per element one add, no multiply
    // (3D rows at pitch tp)
    const unsigned plane = uniform_u32((D == 3) ? (unsigned)(N1 * tp) : (unsigned)N1);
    constexpr int LR = L / RAD;
    const unsigned step = uniform_u32((unsigned)LR * plane);
#pragma unroll
    for (int i = 0; i < E / RAD; ++i) {
        int q, j;
        bmap<L, C, NT, MODE, RAD>(t, i, q, j);
        const int col = min(col0 + q, col0 + nvalid - 1);
        unsigned rowoff;
        if constexpr (D == 3 && HALF) {
            const int k2 = col / N1, k3 = col - (col / N1) * N1;
            rowoff = (unsigned)(min(k2, L - k2) * tp + k3);
        } else if constexpr (D == 3) {
            const int k2 = col / L, k3 = col % L;
            rowoff = (unsigned)(min(k2, L - k2) * tp + min(k3, L - k3));
        } else if constexpr (HALF) {
            rowoff = (unsigned)col;
        } else {
            rowoff = (unsigned)min(col, L - col);
        }
        const unsigned jp = (unsigned)j * plane;
        const unsigned lo = rowoff + jp, hi = rowoff - jp;  // hi wraps; every flat index below is in range
#pragma unroll
        for (int r = 0; r < RAD; ++r) {
            // e = j + r L/R with 0 <= j < L/R: the octant fold min(e, L - e) is
            // e on blocks below L/2 and L - e on blocks at or above it.
            const int e = j + r * LR;
            unsigned flat;
            if ((r + 1) * LR <= L / 2) flat = lo + (unsigned)r * step;
            else if (r * LR >= L / 2) flat = hi + (unsigned)(RAD - r) * step;
            else flat = (unsigned)min(e, L - e) * plane + rowoff;
            if constexpr (CPLX) {
                kt[i * RAD + r] = ld_off<cplx<R>>(table, flat * (unsigned)sizeof(cplx<R>));
            } else {
                kt[i * RAD + r] = mk(ld_off<R>(table, flat * (unsigned)sizeof(R)), R(0));
            }
        }
    }
}

// Staged Khat fetch (3D fused column passes over the octant table, tiles of
// C = 16 or 8 adjacent columns k3 = k3_0 + q of one spectral row k2, k3_0
// and N multiples of C).  The tile needs, for every k1 = 0 .. L/2, C
// consecutive octant entries: k3' = k3_0 .. k3_0 + C - 1, or, for mirrored
// columns (k3_0 >= L/2), k3' = L - k3_0 - (C - 1) .. L - k3_0.  With the row
// pitch a multiple of 16 the first run is one 128-byte line (C = 16) or half
// of one (C = 8); of the second, the first C - 1 entries sit in one line and
// the last (k3' = L - k3_0, a multiple of C) comes from the boundary block,
// where the entries of consecutive k1 are adjacent.  Real tables with C = 8
// (32-byte runs, which cross a line once in four) have no boundary block and
// read the mirrored run in place: the extra request per run measured slower
// there (3D N = 512 Laplace fused pass 2.72 -> 2.75-2.79 ms).  Every entry is loaded once, at the start of the tile (lane c of
// each group of 16 takes run position c), and goes to LDS after the forward
// transform, where each thread picks the values of its spectral indices.
template <int L, int C, int NT>
struct TabStage {
    static_assert((C == 16 || C == 8) && NT % C == 0, "tiles of 16 or 8 columns");
    static constexpr int ROWS = L / 2 + 1;
    static constexpr int N = ROWS * C;
    static constexpr int PER = (N + NT - 1) / NT;
};

template <typename R, int L, int C, int NT, bool CPLX>
__device__ __forceinline__ void tab_stage_issue(cplx<R>* tb, const PassDesc& p, int col0, int t) {
    using TS = TabStage<L, C, NT>;
    constexpr unsigned ES = CPLX ? sizeof(cplx<R>) : sizeof(R);
    const unsigned N1 = (unsigned)p.tabN + 1u, tp = (unsigned)p.tab_pitch, nb = (unsigned)p.tabN / (unsigned)C;
    const int k2 = col0 / L, k3 = col0 % L;
    const unsigned k2f = (unsigned)min(k2, L - k2);
    const bool mir = k3 >= L / 2;
    const int c = t % C;
    const unsigned row0 = (unsigned)(t / C);
    // entry offset of row k1 = row0 + m NT / C: base + m * stride
    unsigned base, stride;
    if ((CPLX || C == 16) && mir && c == C - 1) {
        base = p.tab_bnd + (k2f * nb + (unsigned)(L - k3) / (unsigned)C - 1u) * N1 + row0;
        stride = NT / C;
    } else {
        base = row0 * N1 * tp + k2f * tp + (unsigned)(mir ? L - k3 - (C - 1) : k3) + (unsigned)c;
        stride = (NT / C) * N1 * tp;
    }
#pragma unroll
    for (int m = 0; m < TS::PER; ++m) {
        if (m + 1 < TS::PER || t + m * NT < TS::N) {
            const unsigned off = (base + (unsigned)m * stride) * ES;
            if constexpr (CPLX) tb[m] = ld_off<cplx<R>>(p.table, off);
            else tb[m] = mk(ld_off<R>(p.table, off), R(0));
        }
    }
}

template <typename R, int L, int C, int NT, RP P>
__device__ __forceinline__ void tab_stage_read(const cplx<R>* tb, cplx<R>* kt, cplx<R>* lds, int col0, int t) {
    using TS = TabStage<L, C, NT>;
    constexpr int RAD = P.r[P.n - 1];
    constexpr int E = C * L / NT;
    constexpr int LR = L / RAD;
    const bool mir = (col0 % L) >= L / 2;
    const int c = t % C;
    // entry t + m NT (row (t + m NT) / C, run position c) goes to slot
    // row C + q0: a lane base plus m NT (NT is a multiple of C)
    const int base = (t / C) * C + (mir ? C - 1 - c : c);
#pragma unroll
    for (int m = 0; m < TS::PER; ++m)
        if (m + 1 < TS::PER || t + m * NT < TS::N) lds[base + m * NT] = tb[m];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < E / RAD; ++i) {
        int q, j;
        bmap<L, C, NT, MODE_COL, RAD>(t, i, q, j);
#pragma unroll
        for (int r = 0; r < RAD; ++r) {
            const int e = j + r * LR;
            kt[i * RAD + r] = lds[min(e, L - e) * C + q];
        }
    }
}

// Four-step step B (2D): the spectral index along the axis is k = o + L1 e over
// the whole axis length Lb; the column index folds over Lb as well.
template <typename R, int L, int C, int NT, int MODE, RP P, bool CPLX, bool HALF = false, bool FULL = false>
__device__ __forceinline__ void table_fetch_fs(cplx<R>* kt, const void* __restrict__ table, int tabN, int col0,
                                               int nvalid, int o, int L1, int Lb, int t) {
    constexpr int RAD = P.r[P.n - 1];
    constexpr int E = C * L / NT;
    if constexpr (FULL) {
#pragma unroll
        for (int i = 0; i < E / RAD; ++i) {
            int q, j;
            bmap<L, C, NT, MODE, RAD>(t, i, q, j);
            const unsigned col = (unsigned)min(col0 + q, col0 + nvalid - 1);
#pragma unroll
            for (int r = 0; r < RAD; ++r) {
                const unsigned flat = (unsigned)(o + L1 * (j + r * (L / RAD))) * (unsigned)Lb + col;
                kt[i * RAD + r] = ld_off<cplx<R>>(table, flat * (unsigned)sizeof(cplx<R>));
            }
        }
        return;
    }
    const int N1 = tabN + 1;
#pragma unroll
    for (int i = 0; i < E / RAD; ++i) {
        int q, j;
        bmap<L, C, NT, MODE, RAD>(t, i, q, j);
        const int col = min(col0 + q, col0 + nvalid - 1);
        const unsigned rowoff = HALF ? (unsigned)col : (unsigned)min(col, Lb - col);
#pragma unroll
        for (int r = 0; r < RAD; ++r) {
            const int k = o + L1 * (j + r * (L / RAD));
            const unsigned flat = (unsigned)min(k, Lb - k) * (unsigned)N1 + rowoff;
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
// (four-step step B: the spectral index is o + L1 e over the axis length Lb)
template <typename R, int L, int C, int NT, int MODE, int RAD>
__device__ __forceinline__ void deriv_copy(const cplx<R>* v, cplx<R>* v2, R ks, int t, int o = 0, int L1 = 0,
                                           int Lb = 0) {
    constexpr int E = C * L / NT;
#pragma unroll
    for (int i = 0; i < E / RAD; ++i) {
        int q, j;
        bmap<L, C, NT, MODE, RAD>(t, i, q, j);
#pragma unroll
        for (int r = 0; r < RAD; ++r) {
            const int e = j + r * (L / RAD);
            v2[i * RAD + r] = L1 ? ikap(v[i * RAD + r], o + L1 * e, Lb, ks) : ikap(v[i * RAD + r], e, L, ks);
        }
    }
}

// Real data (real_mode 1 and 2).  A real sequence x of length 2L is read as
// z[m] = x[2m] + i x[2m+1], m < L; with Z = DFT_L(z) and W = e^{-2 pi i/(2L)},
// its spectrum on k in [0, L] is
//   X[k] = (Z[k] + conj Z[L-k])/2 - (i/2) W^k (Z[k] - conj Z[L-k])   (Z L-periodic),
// and conversely the unnormalised inverse of X is recovered from the
// unnormalised length-L inverse of
//   Z'[k] = (X[k] + conj X[L-k]) + i W^-k (X[k] - conj X[L-k]),  k < L,
// whose outputs are (x[2m], x[2m+1]) times 2L.

// After a forward transform (ROW tiles, outputs of plan P in registers):
// the L + 1 values X[k] of every valid pencil, stored with element stride se.
template <typename R, int L, int C, int NT, RP P>
__device__ __forceinline__ void r2c_store(const cplx<R>* v, cplx<R>* lds, cplx<R>* __restrict__ g, const FTile& tl,
                                          long long se, int t, const cplx<R>* __restrict__ tw2) {
    using LY = Lay<L, C, MODE_ROW, (int)sizeof(cplx<R>)>;
    constexpr int RAD = P.r[P.n - 1];
    constexpr int E = C * L / NT;
    constexpr int LR = L / RAD;
#pragma unroll
    for (int i = 0; i < E / RAD; ++i) {
        int q, j;
        bmap<L, C, NT, MODE_ROW, RAD>(t, i, q, j);
#pragma unroll
        for (int r = 0; r < RAD; ++r) lds[LY::idx(q, j + r * LR)] = v[i * RAD + r];
    }
    __syncthreads();
    constexpr int NOUT = C * (L + 1), IT = (NOUT + NT - 1) / NT;
    cplx<R>* __restrict__ gb = g + tl.out0;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int idx = t + it * NT;
        const int q = idx / (L + 1), k = idx - q * (L + 1);
        if (idx < NOUT && q < tl.nvalid) {
            const cplx<R> a = lds[LY::idx(q, k == L ? 0 : k)];
            const cplx<R> b = lds[LY::idx(q, k == 0 ? 0 : L - k)];
            const cplx<R> sm = mk(a.x + b.x, a.y - b.y);  // a + conj b
            const cplx<R> df = mk(a.x - b.x, a.y + b.y);  // a - conj b
            const cplx<R> wd = cmul(tw2[k], df);
            gb[(long long)q * tl.oq + (long long)k * se] = mk(R(0.5) * (sm.x + wd.y), R(0.5) * (sm.y - wd.x));
        }
    }
}

// Before an inverse transform (ROW tiles): the L + 1 inputs X[k] of every
// pencil staged in LDS (q (L + 1) + k), then Z'[e] for this thread's stage-0
// elements e of plan P.
template <typename R, int L, int C, int NT, RP P>
__device__ __forceinline__ void c2r_load(cplx<R>* v, cplx<R>* lds, const cplx<R>* __restrict__ g, const FTile& tl,
                                         long long se, int t, const cplx<R>* __restrict__ tw2) {
    constexpr int RAD = P.r[0];
    constexpr int E = C * L / NT;
    constexpr int LR = L / RAD;
    constexpr int NIN = C * (L + 1), IT = (NIN + NT - 1) / NT;
    constexpr int CHM = sizeof(R) == 8 ? 8 : 16;
    constexpr int CH = IT < CHM ? IT : CHM;  // loads in flight per batch
    const cplx<R>* __restrict__ gb = g + tl.in0;
#pragma unroll
    for (int i0 = 0; i0 < IT; i0 += CH) {
        cplx<R> xin[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int idx = t + (i0 + c) * NT;
            const int q = idx / (L + 1), k = idx - q * (L + 1);
            const int qq = min(q, tl.nvalid - 1);
            if (i0 + c < IT && idx < NIN) xin[c] = gb[(long long)qq * tl.iq + (long long)k * se];
        }
#pragma unroll
        for (int c = 0; c < CH; ++c)
            if (i0 + c < IT && t + (i0 + c) * NT < NIN) lds[t + (i0 + c) * NT] = xin[c];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < E / RAD; ++i) {
        int q, j;
        bmap<L, C, NT, MODE_ROW, RAD>(t, i, q, j);
#pragma unroll
        for (int r = 0; r < RAD; ++r) {
            const int e = j + r * LR;
            const cplx<R> a = lds[q * (L + 1) + e];
            const cplx<R> b = lds[q * (L + 1) + L - e];
            const cplx<R> sm = mk(a.x + b.x, a.y - b.y);
            const cplx<R> df = mk(a.x - b.x, a.y + b.y);
            const cplx<R> cw = cmulc(df, tw2[e]);  // W^-e (a - conj b)
            v[i * RAD + r] = mk(sm.x - cw.y, sm.y + cw.x);
        }
    }
    __syncthreads();
}

enum FastKind : int {
    FK_FWD = 0,
    FK_INV = 1,
    FK_FUSED = 2,
    FK_FUSED_GRAD = 3,
    FK_INV_GRAD = 4,
    FK_INV_DERIV = 5,
    FK_FUSED_DERIV = 6
};

template <int FK>
struct KindIO {
    // forward kinds load zero-padded pencils with the forward plan; inverse
    // kinds load full spectral pencils with the reversed plan
    static constexpr bool fwd_load = FK == FK_FWD || FK == FK_FUSED || FK == FK_FUSED_GRAD || FK == FK_FUSED_DERIV;
};

// Everything after the stage-0 loads of one tile: transforms, multiplies,
// stores.  v holds the stage-0 inputs; kt the Khat values (fused kinds).
// Per-kernel choices, all measured on the 3D N=256 apply (length 512):
//  twl:   the twiddle table (L entries, at most 8 KiB) is copied to LDS once
//         per workgroup; stage twiddles then come from LDS instead of the
//         vector memory path (fused pass 0.47 -> 0.39 ms);
//  split: the fused complex64 length-512 and length-1024 column passes
//         exchange real and imaginary parts in turn through half the LDS (32
//         instead of 64 KiB) and are held to 168 VGPRs, so 3 workgroups share
//         a CU instead of 2 (length 512 at N = 256: 0.39 -> 0.34 ms; length
//         1024 at N = 512: 3.61 -> 3.47 ms); also the complex64 inverse rows
//         of length 8192 (one 64 KiB row per workgroup otherwise; 2D N =
//         4096: 0.136 -> 0.119 ms; the forward rows measured slower split)
//         and of length 512 (21 instead of 38 KiB per workgroup, 4 instead
//         of 2 waves per SIMD: 0.078 -> 0.072 ms at N = 256; the forward
//         rows and the unfused columns of length 512 gain nothing split).
// A row pencil too large for 64 KiB of LDS as complex values (complex128
// rows of length 8192, complex64 rows of 12800) is exchanged as real and
// imaginary parts in turn.
template <typename R, int L, int MODE>
constexpr bool row_needs_split() {
    return MODE == MODE_ROW && L * (int)sizeof(cplx<R>) > 65536;
}

// Wide column tiles: the plain forward and inverse complex64 column passes of
// length 1024 take 16 pencils (128-byte tile rows) through the split
// exchange (64 KiB), instead of the 8 pencils (64-byte rows) of the other
// kinds at that length; see wide_col_C.
template <typename R, int L, int MODE, int FK, int C>
constexpr bool wide_col() {
    return sizeof(R) == 4 && MODE == MODE_COL && L == 1024 && C == 16 && (FK == FK_FWD || FK == FK_INV);
}

template <typename R, int L, int MODE, int FK, int C = 0>
struct Policy {
    static constexpr bool twl = L * (int)sizeof(cplx<R>) <= 8192 && make_plan(L, kMaxRad<R>).n >= 2;
    static constexpr bool wide = wide_col<R, L, MODE, FK, C>();
    static constexpr bool split =
        (sizeof(R) == 4 && MODE == MODE_COL && (FK == FK_FUSED || FK == FK_FUSED_DERIV) && (L == 512 || L == 1024)) ||
        (sizeof(R) == 4 && MODE == MODE_ROW && FK == FK_INV && (L == 512 || L >= 8192)) || wide ||
        row_needs_split<R, L, MODE>();
    // the two-output kinds (two spectra per thread) keep the default budget;
    // wide tiles (8 waves) fit two workgroups per CU at 4 waves per SIMD
    static constexpr int min_waves =
        wide ? 4 : ((split && sizeof(R) == 4 && FK != FK_INV_GRAD && FK != FK_FUSED_GRAD) ? 3 : 1);
};

// The C2R rows (FS & 7 == 4) stage whole complex values in LDS and keep the
// plain exchange.
template <typename R, int L, int MODE, int FK, int FS, int C = 0>
constexpr bool use_split() {
    // plain complex64 forward rows of length >= 8192 split as well (2D N = 4096:
    // 0.091 -> 0.085 ms once the stage twiddles sit in LDS; with them in
    // global memory the split rows had measured slower)
    constexpr bool fwd_rows = sizeof(R) == 4 && MODE == MODE_ROW && FK == FK_FWD && L >= 8192 && FS == 0;
    // plain complex64 rows of length 1024: 25 instead of 42 KiB per 2-wave
    // workgroup, 12 instead of 6 waves per CU (3D N = 512: forward rows
    // 0.614 -> 0.586 ms, inverse 0.615 -> 0.555 ms; 2D N = 512, whose 128 row
    // tiles do not fill the chip anyway, +0.4 us); the two-output inverse
    // rows of the gradient (256 VGPRs) 6 -> 8 waves per CU (3D N = 512
    // gradient 12.95 -> 12.54 ms).  Not the real-data rows (FS & 7 = 3, 4),
    // whose pre- and post-processing reads the whole complex pencil from LDS.
    constexpr bool rows1024 = sizeof(R) == 4 && MODE == MODE_ROW && L == 1024 && FS == 0 &&
                              (FK == FK_FWD || FK == FK_INV || FK == FK_INV_GRAD);
    return (Policy<R, L, MODE, FK, C>::split && ((FS & 7) != 4 || row_needs_split<R, L, MODE>())) || fwd_rows ||
           rows1024;
}
template <typename R, int L, int MODE, int FK, int FS, int C = 0>
constexpr int kernel_waves() {
    // split plain rows (the two-output kind keeps its two spectra in registers)
    if constexpr (!Policy<R, L, MODE, FK, C>::split && use_split<R, L, MODE, FK, FS, C>())
        return FK == FK_INV_GRAD ? 2 : 3;
    else return use_split<R, L, MODE, FK, FS, C>() ? Policy<R, L, MODE, FK, C>::min_waves : 1;
}

// FS: 0 plain pass; 1 four-step step A (forward, outputs times W^{o e});
// 2 four-step step B (full-length forward, Khat at index o + L1 e, full-length
// inverse, outputs times conj W^{o e}).
template <typename R, int L, int C, int NT, int MODE, int FK, int D, bool CPLX, int FS>
__device__ __forceinline__ void tile_body(cplx<R>* v, cplx<R>* kt, cplx<R>* lds, const FTile& tl,
                                          const PassDesc& p, int t, const cplx<R>* tw) {
    constexpr int FSB = FS & 7;
    constexpr int NOUTI = FSB == 2 ? L : L / 2;  // inverse outputs kept
    constexpr int PTI = FSB == 2 ? 2 : 0;        // post twiddle of inverse outputs
    constexpr RP F = make_plan(L, kMaxRad<R>);
    constexpr RP I = reversed(F);
    constexpr int E = C * L / NT;
    constexpr bool SP = use_split<R, L, MODE, FK, FS, C>();
    cplx<R>* __restrict__ gout = reinterpret_cast<cplx<R>*>(p.out);
    cplx<R>* __restrict__ gout2 = reinterpret_cast<cplx<R>*>(p.out2);
    const R ks = (R)p.kscale;
    if constexpr (FK == FK_FWD && FSB == 3) {
        static_assert(!SP, "the real-output post-processing reads whole complex values from LDS");
        run_from<R, L, C, NT, MODE, -1, F, 0, SP>(v, lds, t, tw);
        r2c_store<R, L, C, NT, F>(v, lds, gout, tl, p.out_se, t, reinterpret_cast<const cplx<R>*>(p.tw_big));
    } else if constexpr (FK == FK_FWD) {
        run_from<R, L, C, NT, MODE, -1, F, 0, SP>(v, lds, t, tw);
        store_global<R, L, C, NT, MODE, F, L, FSB == 1 ? 1 : 0>(v, gout, tl, p.out_se, t, p.tw_big);
    } else if constexpr (FK == FK_INV || FK == FK_INV_DERIV) {
        if constexpr (FK == FK_INV_DERIV) {
            cplx<R> w[E];
            deriv_copy<R, L, C, NT, MODE, I.r[0]>(v, w, ks, t);
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = w[e];
        }
        run_from<R, L, C, NT, MODE, +1, I, 0, SP>(v, lds, t, tw);
        store_global<R, L, C, NT, MODE, I, L / 2>(v, gout, tl, p.out_se, t);
    } else if constexpr (FK == FK_INV_GRAD) {
        cplx<R> w[E];
        deriv_copy<R, L, C, NT, MODE, I.r[0]>(v, w, ks, t);
        run_from<R, L, C, NT, MODE, +1, I, 0, SP>(v, lds, t, tw);
        store_global<R, L, C, NT, MODE, I, L / 2>(v, gout, tl, p.out_se, t);
        __syncthreads();
        run_from<R, L, C, NT, MODE, +1, I, 0, SP>(w, lds, t, tw);
        store_global<R, L, C, NT, MODE, I, L / 2>(w, gout2, tl, p.out_se, t);
    } else {
        // exchange padding (ColPad) in the plain fused kind only
        constexpr bool CPD = FK == FK_FUSED && FS == 0;
        run_from<R, L, C, NT, MODE, -1, F, 0, SP, CPD>(v, lds, t, tw);
        table_apply<R, E, CPLX>(v, kt);
        if constexpr (FK == FK_FUSED_DERIV) {
            if constexpr (FSB == 2) deriv_copy<R, L, C, NT, MODE, F.r[F.n - 1]>(v, v, ks, t, tl.o, p.fs_L1, p.L_big);
            else deriv_copy<R, L, C, NT, MODE, F.r[F.n - 1]>(v, v, ks, t);
        }
        if constexpr (FK == FK_FUSED || FK == FK_FUSED_DERIV) {
            run_from<R, L, C, NT, MODE, +1, I, 0, SP, CPD>(v, lds, t, tw);
            store_global<R, L, C, NT, MODE, I, NOUTI, PTI>(v, gout, tl, p.out_se, t, p.tw_big);
        } else {
            cplx<R> w[E];
            if constexpr (FSB == 2) deriv_copy<R, L, C, NT, MODE, F.r[F.n - 1]>(v, w, ks, t, tl.o, p.fs_L1, p.L_big);
            else deriv_copy<R, L, C, NT, MODE, F.r[F.n - 1]>(v, w, ks, t);
            run_from<R, L, C, NT, MODE, +1, I, 0, SP>(v, lds, t, tw);
            store_global<R, L, C, NT, MODE, I, NOUTI, PTI>(v, gout, tl, p.out_se, t, p.tw_big);
            __syncthreads();
            run_from<R, L, C, NT, MODE, +1, I, 0, SP>(w, lds, t, tw);
            store_global<R, L, C, NT, MODE, I, NOUTI, PTI>(w, gout2, tl, p.out_se, t, p.tw_big);
        }
    }
}

// One tile (tile index b of the pass described by p).
template <typename R, int L, int C, int NT, int MODE, int FK, int D, bool CPLX, int FS>
__device__ __forceinline__ void fast_run(const PassDesc& p, unsigned b) {
    using PO = Policy<R, L, MODE, FK, C>;
    constexpr RP F = make_plan(L, kMaxRad<R>);
    constexpr RP I = reversed(F);
    constexpr int E = C * L / NT;
    constexpr bool FL = KindIO<FK>::fwd_load;
    constexpr RP PL = FL ? F : I;
    constexpr int FSB = FS & 7;
    constexpr bool HALF = (FS & 8) != 0;
    constexpr bool FULL = (FS & 16) != 0;
    constexpr int NIN = (FL && FSB != 2) ? L / 2 : L;
    using LY = Lay<L, C, MODE, (int)sizeof(cplx<R>), use_split<R, L, MODE, FK, FS, C>() ? 65536 : kPadLimit>;
    constexpr int LYP = LY::size + ((MODE == MODE_COL && FK == FK_FUSED && FS == 0) ? col_pad_slots<L, C, F>() : 0);
    constexpr int NLDS0 = use_split<R, L, MODE, FK, FS, C>() ? (LYP + 1) / 2 : LYP;
    // staged Khat fetch: plain fused and fused-derivative complex64 columns of
    // the staged lengths (derivative kind at 3D N = 512: 0.15 ms per gradient)
    constexpr bool STG = (FK == FK_FUSED || FK == FK_FUSED_DERIV) && FSB == 0 && !HALF && !FULL &&
                         MODE == MODE_COL && D == 3 && sizeof(R) == 4 && C == staged_fetch_C(L);
    constexpr int NLDS1 = (FSB == 4 && C * (L + 1) > NLDS0) ? C * (L + 1) : NLDS0;
    constexpr int NSTG = STG ? (L / 2 + 1) * C : 0;  // TabStage::N
    constexpr int NLDS = NSTG > NLDS1 ? NSTG : NLDS1;
    __shared__ cplx<R> lds[NLDS];
    __shared__ cplx<R> twl[PO::twl ? L : 1];
    const cplx<R>* __restrict__ tw = reinterpret_cast<const cplx<R>*>(p.tw);
    constexpr bool TWS = tw_split<R, L>();
    __shared__ cplx<R> tws[TWS ? 64 + L / 64 : 1];
    if constexpr (PO::twl) {
        // copied once per workgroup; first read after the barrier of the
        // first exchange (stage 0 of every plan runs without twiddles)
        for (int i = threadIdx.x; i < L; i += NT) twl[i] = tw[i];
        tw = twl;
    } else if constexpr (TWS) {
        for (int i = threadIdx.x; i < 64 + L / 64; i += NT) tws[i] = tw[i < 64 ? i : (i - 64) * 64];
        tw = tws;
    }
    const int t = threadIdx.x;
    const FTile tl = fast_tile<C, MODE>(p, b);
    const cplx<R>* __restrict__ gin = reinterpret_cast<const cplx<R>*>(p.in);
    cplx<R> v[E];
    constexpr bool TAB = FK == FK_FUSED || FK == FK_FUSED_GRAD || FK == FK_FUSED_DERIV;
    cplx<R> kt[TAB ? E : 1];
    if constexpr (FSB == 4) {
        static_assert(MODE == MODE_ROW && FK == FK_INV, "real-output pre-processing is a row inverse");
        c2r_load<R, L, C, NT, PL>(v, lds, gin, tl, p.in_se, t, reinterpret_cast<const cplx<R>*>(p.tw_big));
    } else {
        cplx<R> vn[LoadSet<R, L, C, NT, PL, NIN>::NV];
        issue_loads<R, L, C, NT, MODE, PL, NIN>(vn, gin, tl, p.in_se, t);
        if constexpr (STG) {
            // the tile's table entries wait in tb until the forward transform
            // is done (the dispatcher checks that the table has the boundary block)
            constexpr bool SP = use_split<R, L, MODE, FK, FS, C>();
            cplx<R> tb[TabStage<L, C, NT>::PER];
            tab_stage_issue<R, L, C, NT, CPLX>(tb, p, tl.col0, t);
            expand<R, L, C, NT, PL, NIN>(v, vn);
            constexpr bool CPD = FK == FK_FUSED;  // exchange padding: plain fused kind only
            run_from<R, L, C, NT, MODE, -1, F, 0, SP, CPD>(v, lds, t, tw);
            tab_stage_read<R, L, C, NT, F>(tb, kt, lds, tl.col0, t);
            table_apply<R, E, CPLX>(v, kt);
            if constexpr (FK == FK_FUSED_DERIV) deriv_copy<R, L, C, NT, MODE, F.r[F.n - 1]>(v, v, (R)p.kscale, t);
            __syncthreads();  // the inverse's first exchange overwrites the staged entries
            run_from<R, L, C, NT, MODE, +1, I, 0, SP, CPD>(v, lds, t, tw);
            store_global<R, L, C, NT, MODE, I, L / 2>(v, reinterpret_cast<cplx<R>*>(p.out), tl, p.out_se, t);
            return;
        }
        if constexpr (TAB && FSB == 2)
            table_fetch_fs<R, L, C, NT, MODE, F, CPLX, HALF, FULL>(kt, p.table, p.tabN, tl.col0, tl.nvalid, tl.o,
                                                                   p.fs_L1, p.L_big, t);
        else if constexpr (TAB)
            table_fetch<R, L, C, NT, MODE, F, D, CPLX, HALF, FULL>(kt, p.table, p.tabN, p.tab_pitch, tl.col0,
                                                                tl.nvalid, t);
        expand<R, L, C, NT, PL, NIN>(v, vn);
    }
    tile_body<R, L, C, NT, MODE, FK, D, CPLX, FS>(v, kt, lds, tl, p, t, tw);
}

// Mirror-paired tile order of the fused column passes over the octant table:
// the table value of column (k2, k3) is shared by (L - k2, k3), (k2, L - k3)
// and (L - k2, L - k3), so those tiles are placed next to each other in the
// launch order (and hence on one XCD, close in time): spectral row k2 runs
// in the order 0, 1, L-1, 2, L-2, ..., L/2 and the L/C tiles of a row in the
// order 0, L/C-1, 1, L/C-2, ...  Both maps are bijections.  Measured on the
// 3D N = 256 apply: fused pass 0.345 -> 0.330 ms.
__device__ __forceinline__ unsigned mirror_row(unsigned i, unsigned n) {
    if (i == 0) return 0;
    if (i == n - 1) return n / 2;
    const unsigned m = (i + 1) / 2;
    return (i & 1u) ? m : n - m;
}
__device__ __forceinline__ unsigned mirror_tile(unsigned s, unsigned n) { return (s & 1u) ? n - 1 - (s >> 1) : (s >> 1); }

template <int L, int C, int MODE, int FK, int D, int FS>
__device__ __forceinline__ unsigned tile_order(const PassDesc& p, unsigned b) {
    constexpr bool TAB = FK == FK_FUSED || FK == FK_FUSED_GRAD || FK == FK_FUSED_DERIV;
    if constexpr (TAB && MODE == MODE_COL && FS == 0 && L % C == 0) {
        constexpr unsigned nt = L / C;
        if (D == 3 && p.inner == L * L) return mirror_row(b / nt, L) * nt + mirror_tile(b % nt, nt);
        if (D == 2 && p.inner == L) return (b / nt) * nt + mirror_tile(b % nt, nt);
    }
    return b;
}

// One tile per workgroup.
template <typename R, int L, int C, int NT, int MODE, int FK, int D, bool CPLX, int FS>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(kernel_waves<R, L, MODE, FK, FS, C>())))
fast_kernel(PassDesc p) {
    unsigned b = blockIdx.x;
    if constexpr ((FK == FK_FUSED || FK == FK_FUSED_DERIV || FK == FK_FUSED_GRAD) && (FS & 7) == 2 && (FS & 16) == 0 &&
                  MODE == MODE_COL) {
        // four-step step B (2D, octant table): tile (k1 = o, column block).
        // Spectral index o + L1 e mirrors to (L1 - o) + L1 (L2 - 1 - e) and
        // column c to 2N - c, so tiles o and L1 - o, and mirrored column
        // blocks, read the same table entries: launch them next to each
        // other, in launch order (2D N = 4096: 0.246 -> 0.231 ms; with the
        // XCD-grouped order 0.237 ms)
        const unsigned nt = (unsigned)((p.inner + C - 1) / C);
        const unsigned no = (unsigned)p.outer;
        if (nt * no == gridDim.x && (no & 1u) == 0u && (nt & 1u) == 0u)
            b = mirror_row(b / nt, no) * nt + mirror_tile(b % nt, nt);
    } else if (p.xcd_map) {
        b = tile_order<L, C, MODE, FK, D, FS>(p, xcd_tile(b, gridDim.x));
    }
    fast_run<R, L, C, NT, MODE, FK, D, CPLX, FS>(p, b);
}

// Grouped launch: the same pass over several independent arrays (one
// descriptor each, same length and kind); item i owns the workgroups
// [starts[i], starts[i + 1]).
template <typename R, int L, int C, int NT, int MODE, int FK, int D, bool CPLX, int FS>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(kernel_waves<R, L, MODE, FK, FS, C>())))
fast_group_kernel(const PassDesc* __restrict__ descs, const unsigned* __restrict__ starts, int nitems) {
    const unsigned b = xcd_tile(blockIdx.x, gridDim.x);
    int i = 0;
    while (i + 1 < nitems && b >= starts[i + 1]) ++i;
    fast_run<R, L, C, NT, MODE, FK, D, CPLX, FS>(descs[i], b - starts[i]);
}

// --------------------------------------------------------------- dispatch --
template <typename R, int L, int C, int NT, int MODE, int FK, int D, bool CPLX, int FS = 0, bool GROUP = false>
hipError_t launch_k(const PassDesc& p, long long ntiles, hipStream_t s, const GroupArgs* g) {
    if constexpr (GROUP) {
        hipLaunchKernelGGL((fast_group_kernel<R, L, C, NT, MODE, FK, D, CPLX, FS>), dim3(g->ntiles), dim3(NT), 0, s,
                           g->descs, g->starts, g->nitems);
    } else {
        hipLaunchKernelGGL((fast_kernel<R, L, C, NT, MODE, FK, D, CPLX, FS>), dim3((unsigned)ntiles), dim3(NT), 0, s, p);
    }
    return hipGetLastError();
}

template <typename R, int L, int C, int NT, int MODE, bool GROUP>
hipError_t launch_shape(const PassDesc& p, int kind, hipStream_t s, const GroupArgs* ga) {
    long long nblocks = GROUP ? (long long)ga->ntiles
                              : (MODE == MODE_COL ? (long long)p.outer * ((p.inner + C - 1) / C) : (p.outer + C - 1) / C);
    if (nblocks <= 0) return hipSuccess;
    if (nblocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    const bool fused = kind == KIND_FUSED || kind == KIND_FUSED_GRAD || kind == KIND_FUSED_DERIV;
    if (p.real_mode) {
        // real-data variants: rows in and out of the half spectrum, and the
        // fused pass on a half spectrum (apply only; real tables)
        if constexpr (MODE == MODE_ROW) {
            // no real-data rows where one complex pencil needs the split
            // exchange (their C2R staging holds L + 1 whole values)
            if constexpr (L * (int)sizeof(cplx<R>) <= 65536) {
                if (p.real_mode == 1 && kind == KIND_FWD) return launch_k<R, L, C, NT, MODE, FK_FWD, 3, false, 3, GROUP>(p, nblocks, s, ga);
                if (p.real_mode == 2 && kind == KIND_INV) return launch_k<R, L, C, NT, MODE, FK_INV, 3, false, 4, GROUP>(p, nblocks, s, ga);
            }
        } else {
            if (p.real_mode == 4 && kind == KIND_FUSED && !p.table_complex) {
                if (p.fs_L1 && p.d == 2 && p.post_tw == 2)
                    return launch_k<R, L, C, NT, MODE, FK_FUSED, 2, false, 2 | 8, GROUP>(p, nblocks, s, ga);
                if (!p.fs_L1 && p.d == 3) return launch_k<R, L, C, NT, MODE, FK_FUSED, 3, false, 8, GROUP>(p, nblocks, s, ga);
                if (!p.fs_L1 && p.d == 2) return launch_k<R, L, C, NT, MODE, FK_FUSED, 2, false, 8, GROUP>(p, nblocks, s, ga);
            }
        }
        return hipErrorInvalidValue;
    }
    if constexpr (MODE == MODE_ROW) {
        if (fused) return hipErrorInvalidValue;  // fused passes are column passes
    } else if (fused) {
        // D (table dimension), CPLX (table type) and FS (four-step step B) are compile-time
        auto by_kind = [&](auto dc, auto cc, auto fc) -> hipError_t {
            constexpr int DD = decltype(dc)::value;
            constexpr bool CC = decltype(cc)::value;
            constexpr int FF = decltype(fc)::value;
            if (kind == KIND_FUSED_GRAD) return launch_k<R, L, C, NT, MODE, FK_FUSED_GRAD, DD, CC, FF, GROUP>(p, nblocks, s, ga);
            if (kind == KIND_FUSED_DERIV) return launch_k<R, L, C, NT, MODE, FK_FUSED_DERIV, DD, CC, FF, GROUP>(p, nblocks, s, ga);
            return launch_k<R, L, C, NT, MODE, FK_FUSED, DD, CC, FF, GROUP>(p, nblocks, s, ga);
        };
        using I2 = std::integral_constant<int, 2>;
        using I3 = std::integral_constant<int, 3>;
        using I0 = std::integral_constant<int, 0>;
        using T_ = std::true_type;
        using F_ = std::false_type;
        if (p.table_full) {
            // full complex table (convection kernel)
            if (!p.table_complex) return hipErrorInvalidValue;
            if (p.fs_L1) {
                if (p.d != 2 || p.post_tw != 2) return hipErrorInvalidValue;
                return by_kind(I2{}, T_{}, std::integral_constant<int, 2 | 16>{});
            }
            if (p.d == 3) return by_kind(I3{}, T_{}, std::integral_constant<int, 16>{});
            return by_kind(I2{}, T_{}, std::integral_constant<int, 16>{});
        }
        if (p.fs_L1) {
            // four-step step B (2D only)
            if (p.d != 2 || p.post_tw != 2) return hipErrorInvalidValue;
            return p.table_complex ? by_kind(I2{}, T_{}, I2{}) : by_kind(I2{}, F_{}, I2{});
        }
        // the staged fetch of plain fused passes needs the table's boundary block
        if (sizeof(R) == 4 && staged_fetch_C(L) == C && (C == 16 || p.table_complex) && p.d == 3 &&
            (kind == KIND_FUSED || kind == KIND_FUSED_DERIV) && !p.tab_bnd)
            return hipErrorInvalidValue;
        if (p.d == 3) return p.table_complex ? by_kind(I3{}, T_{}, I0{}) : by_kind(I3{}, F_{}, I0{});
        return p.table_complex ? by_kind(I2{}, T_{}, I0{}) : by_kind(I2{}, F_{}, I0{});
    }
    if (p.post_tw || p.fs_L1) {
        // four-step step A (column forward with post twiddle)
        if constexpr (MODE == MODE_COL) {
            if (kind == KIND_FWD && p.post_tw == 1 && !p.fs_L1)
                return launch_k<R, L, C, NT, MODE, FK_FWD, 3, false, 1, GROUP>(p, nblocks, s, ga);
        }
        return hipErrorInvalidValue;
    }
    switch (kind) {
        case KIND_FWD: return launch_k<R, L, C, NT, MODE, FK_FWD, 3, false, 0, GROUP>(p, nblocks, s, ga);
        case KIND_INV: return launch_k<R, L, C, NT, MODE, FK_INV, 3, false, 0, GROUP>(p, nblocks, s, ga);
        case KIND_INV_GRAD: return launch_k<R, L, C, NT, MODE, FK_INV_GRAD, 3, false, 0, GROUP>(p, nblocks, s, ga);
        case 100 + KIND_INV: return launch_k<R, L, C, NT, MODE, FK_INV_DERIV, 3, false, 0, GROUP>(p, nblocks, s, ga);
        default: return hipErrorInvalidValue;
    }
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
    const RP p = make_plan(L, esize == 8 ? 32 : 16);
    int lc = 1;
    for (int i = 0; i < p.n; ++i) lc = lc / gcd_i(lc, p.r[i]) * p.r[i];
    // elements per thread: at least 32 complex64 (16 complex128) values, for
    // butterfly-level parallelism in a thread, except complex64 lengths 96 to
    // 256 (the 3D N = 48..128 grids), where 16 gives twice the waves and
    // measured faster (3D N = 128 apply 0.115 -> 0.101 ms, N = 64 0.034 ->
    // 0.029 ms; the 64-density batch 2.48 -> 2.39 ms); shorter lengths (the
    // four-step pieces of 2D N = 1024) measured slower with 16
    const int target = esize == 16 ? 16 : ((L >= 96 && L <= 256) ? 16 : 32);
    const int E = lc >= target ? lc : (target / lc) * lc;
    const int LP = mode == MODE_COL ? L : L + L / 16;
    // rows whose single pencil exceeds 64 KiB exchange half values (split)
    const int les = (mode == MODE_ROW && L * esize > 65536) ? esize / 2 : esize;
    int C = mode == MODE_COL ? 16 : 8;
    // length-400 columns (3D N = 200) take 8 pencils: 16-pencil tiles (53 KiB
    // of LDS, 5 waves) leave room for 2 workgroups per CU, 8-pencil tiles for
    // 4 (fused pass 0.39 -> 0.25 ms, apply 0.64 -> 0.47 ms); length 500
    // measured slower with 8 (apply 1.04 -> 1.20 ms: 4 waves for 3.1 waves'
    // work, 64-byte runs)
    if (mode == MODE_COL && L == 400) C = 8;
    // complex64 rows of length 300 take 16 pencils (160 threads, 40 KiB of
    // LDS) instead of 8 (80 threads, a quarter-full second wave): 3D N = 150
    // apply 0.304 -> 0.296 ms
    if (mode == MODE_ROW && L == 300 && esize == 8) C = 16;
    while (C > 1 && C * LP * les > 65536) C /= 2;
    if (C * LP * les > 65536 && L * les > 65536) return Shape{0, E, 0};  // one pencil does not fit
    while (C * L / E < 64 && C < 64 && 2 * C * LP * les <= 65536) C *= 2;
    if (C * L / E < 64) return Shape{0, E, 0};  // under one wave: left to the generic kernel
    return Shape{C, E, C * L / E};
}

// ROWS_ONLY: long lengths are instantiated for row passes only (their column
// passes use the four-step decomposition).
template <typename R, int L, int MODE, bool GROUP>
hipError_t launch_len_mode(const PassDesc& p, int kind, hipStream_t s, const GroupArgs* ga) {
    constexpr Shape S = shape_for(L, MODE, (int)sizeof(cplx<R>));
    if constexpr (wide_col<R, L, MODE, FK_FWD, 16>()) {
        // wide column tiles (plain forward / inverse passes only)
        if (p.C == 16) {
            constexpr int C = 16, NT = C * L / S.E;
            if (p.real_mode || p.post_tw || p.fs_L1 || (kind != KIND_FWD && kind != KIND_INV))
                return hipErrorInvalidValue;
            const long long nblocks = GROUP ? (long long)ga->ntiles : (long long)p.outer * ((p.inner + C - 1) / C);
            if (nblocks <= 0) return hipSuccess;
            if (nblocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
            if (kind == KIND_FWD) return launch_k<R, L, C, NT, MODE, FK_FWD, 3, false, 0, GROUP>(p, nblocks, s, ga);
            return launch_k<R, L, C, NT, MODE, FK_INV, 3, false, 0, GROUP>(p, nblocks, s, ga);
        }
    }
    if constexpr (S.C == 0) {
        return hipErrorInvalidValue;
    } else {
        static_assert(S.C * L % S.E == 0 && S.NT >= 64 && S.NT <= 1024, "bad launch shape");
        if (p.C != S.C) return hipErrorInvalidValue;
        return launch_shape<R, L, S.C, S.NT, MODE, GROUP>(p, kind, s, ga);
    }
}

template <typename R, int L, bool ROWS_ONLY, bool GROUP = false>
hipError_t launch_len(const PassDesc& p, int mode, int kind, hipStream_t s, const GroupArgs* ga = nullptr) {
    if (mode == MODE_ROW) return launch_len_mode<R, L, MODE_ROW, GROUP>(p, kind, s, ga);
    if constexpr (ROWS_ONLY) return hipErrorInvalidValue;
    else return launch_len_mode<R, L, MODE_COL, GROUP>(p, kind, s, ga);
}

// Whether the 32-bit lane offsets of the specialised kernel cover a pass
// with these strides (element units): lane part (q iq + j se) * size, with
// j below L / (radix of the loading or storing stage).
template <typename R, int L, int MODE>
bool offsets_fit(long long in_se, long long out_se, long long in_iq, long long out_iq) {
    constexpr RP F = make_plan(L, kMaxRad<R>);
    constexpr RP I = reversed(F);
    constexpr Shape S = shape_for(L, MODE, (int)sizeof(cplx<R>));
    if constexpr (S.C == 0) {
        return false;
    } else {
        const int rl = F.r[0] < I.r[0] ? F.r[0] : I.r[0];
        const int rs = F.r[F.n - 1] < I.r[I.n - 1] ? F.r[F.n - 1] : I.r[I.n - 1];
        const long double es = (long double)sizeof(cplx<R>);
        const long double lim = 4294967296.0L;
        const long double a = ((long double)(S.C - 1) * in_iq + (long double)(L / rl - 1) * in_se) * es;
        const long double b = ((long double)(S.C - 1) * out_iq + (long double)(L / rs - 1) * out_se) * es;
        return a < lim && b < lim;
    }
}

template <typename R, int L, bool ROWS_ONLY>
bool fits(int mode, long long in_se, long long out_se, long long in_iq, long long out_iq) {
    if (mode == MODE_ROW) return offsets_fit<R, L, MODE_ROW>(in_se, out_se, in_iq, out_iq);
    if constexpr (ROWS_ONLY) return false;
    else return offsets_fit<R, L, MODE_COL>(in_se, out_se, in_iq, out_iq);
}

template <typename R, int L, bool ROWS_ONLY>
int shape_C(int mode) {
    if (mode == MODE_COL && ROWS_ONLY) return 0;
    return mode == MODE_COL ? shape_for(L, MODE_COL, (int)sizeof(cplx<R>)).C
                            : shape_for(L, MODE_ROW, (int)sizeof(cplx<R>)).C;
}

}  // namespace fastfft

// One translation unit per length instantiates these through
// VG_FAST_INSTANTIATE(L); fft_fast.hip dispatches on the length.
#define VG_FAST_INSTANTIATE(LL, ROWS_ONLY)                                                                   \
    int fast_C_##LL(int mode, bool fp64) {                                                                   \
        return fp64 ? fastfft::shape_C<double, LL, ROWS_ONLY>(mode) : fastfft::shape_C<float, LL, ROWS_ONLY>(mode); \
    }                                                                                                        \
    bool fast_fits_##LL(int mode, bool fp64, long long ise, long long ose, long long iiq, long long oiq) {  \
        return fp64 ? fastfft::fits<double, LL, ROWS_ONLY>(mode, ise, ose, iiq, oiq)                          \
                    : fastfft::fits<float, LL, ROWS_ONLY>(mode, ise, ose, iiq, oiq);                           \
    }                                                                                                        \
    hipError_t launch_fast_##LL(const PassDesc& p, int mode, int kind, bool fp64, hipStream_t s) {           \
        return fp64 ? fastfft::launch_len<double, LL, ROWS_ONLY>(p, mode, kind, s)                           \
                    : fastfft::launch_len<float, LL, ROWS_ONLY>(p, mode, kind, s);                           \
    }

// Grouped launches (one translation unit per length, separate from the
// single-array kernels so that both compile in parallel).
#define VG_FAST_GROUP_INSTANTIATE(LL)                                                                        \
    hipError_t launch_fast_group_##LL(const PassDesc& proto, const GroupArgs& g, int mode, int kind, bool fp64, \
                                      hipStream_t s) {                                                       \
        return fp64 ? fastfft::launch_len<double, LL, false, true>(proto, mode, kind, s, &g)                 \
                    : fastfft::launch_len<float, LL, false, true>(proto, mode, kind, s, &g);                 \
    }

}  // namespace vg
