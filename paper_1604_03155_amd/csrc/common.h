// Internal declarations shared by the HIP kernels and the host runtime of the
// volume-potential library.  Not part of the public ABI (include/vg.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

namespace vg {

// ---------------------------------------------------------------- complex --
template <typename R>
struct alignas(2 * sizeof(R)) cplx {
    R x, y;
};
using c32 = cplx<float>;
using c64 = cplx<double>;

template <typename R>
__host__ __device__ __forceinline__ cplx<R> mk(R a, R b) {
    cplx<R> c;
    c.x = a;
    c.y = b;
    return c;
}
template <typename R>
__host__ __device__ __forceinline__ cplx<R> operator+(cplx<R> a, cplx<R> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename R>
__host__ __device__ __forceinline__ cplx<R> operator-(cplx<R> a, cplx<R> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename R>
__host__ __device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
    return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename R>
__host__ __device__ __forceinline__ cplx<R> cmulc(cplx<R> a, cplx<R> b) {
    return mk(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename R>
__host__ __device__ __forceinline__ cplx<R> scale(cplx<R> a, R s) { return mk(a.x * s, a.y * s); }

// ------------------------------------------------------------ FFT passes --
// A pass runs one batched 1D FFT along one axis of a strided array.  Pencils
// (1D lines along the axis) are identified by (o, c): outer block o and
// column c.  Element e of pencil (o, c) lives at  o*so + c + e*se  (element
// units) for column passes, and at  o*so + e  for row passes (contiguous
// axis, one column).
enum PassMode : int { MODE_ROW = 0, MODE_COL = 1 };

// What a pass does between load and store.
enum PassKind : int {
    KIND_FWD = 0,        // forward DFT (exponent sign -)
    KIND_INV = 1,        // inverse DFT (sign +), unnormalised
    KIND_FUSED = 2,      // forward, multiply by the Khat octant, inverse
    KIND_FUSED_GRAD = 3, // as FUSED, second output multiplied by i*kappa along this axis
    KIND_INV_GRAD = 4,   // inverse to out, and inverse of (i*kappa * in) to out2
    KIND_FUSED_DERIV = 5,  // forward, multiply by the Khat octant and i*kappa, inverse
};

constexpr int kMaxStages = 12;

struct PassDesc {
    const void* in;
    void* out;
    void* out2;             // second output (gradient kinds)
    const void* tw;         // twiddles e^{-2 pi i t / L}, t in [0, L)
    const void* table;      // Khat octant (fused kinds), already divided by (2N)^d
    long long in_so, out_so;  // outer strides (elements)
    long long in_se, out_se;  // axis strides (elements)
    int L;                  // transform length
    int n_in;               // inputs e >= n_in are zero (pruned zero padding)
    int n_out;              // only outputs e < n_out are stored (crop)
    int inner;              // columns per outer block (MODE_COL); 1 for rows
    int outer;              // outer blocks (MODE_COL) or pencils (MODE_ROW)
    int C;                  // pencils per workgroup
    int specialised;        // 1: run the length-specialised kernel (chosen at plan time)
    int nst;
    int radix[kMaxStages];
    // Khat octant indexing for fused kinds: the pencil's other spectral
    // indices come from its column: d == 3: c = k2 * (2N) + k3; d == 2: c = k2.
    int d;
    int tabN;               // N of the plan (octant is (N+1)^d)
    // 3D octant tables: entries between consecutive (k1, k2) rows, N + 1
    // rounded up to a multiple of 16 (N >= 96) so that runs of 16 entries
    // starting at k3 = 16 m are whole 128-byte lines (complex64); 2D tables
    // and 3D N < 96: N + 1
    int tab_pitch;
    // staged table fetch (3D FP32, C = staged_fetch_C(2N) > 0; C = 8: complex
    // tables only): element offset in `table` of the boundary block, which
    // repeats the entries k3 = C (b + 1), b < N / C, of every row in the
    // order [k2][b][k1]; 0 when absent
    unsigned tab_bnd;
    int table_complex;      // 0: real table (Laplace), 1: complex
    // spectral derivative along this pass's axis (gradient kinds): i*kappa,
    // kappa = kscale * signed(k), zero at the Nyquist index k = Laxis/2.
    double kscale;
    // Four-step passes (an axis of length L_big = L1 * L2 done as length-L1
    // and length-L2 transforms).  post_tw: stored outputs are multiplied by
    // W_{L_big}^{o e} (1) or its conjugate (2), o the pencil's outer index and
    // e the output index.  fs_L1: the spectral index along the axis is
    // o + fs_L1 * e (0: it is e).
    const void* tw_big;
    int L_big;
    int post_tw;
    int fs_L1;
    // specialised kernels: 1 maps workgroup slots to tiles XCD by XCD (each
    // of the 8 XCDs gets a contiguous range of tiles), 0 keeps launch order
    int xcd_map;
    // real-data passes (specialised kernels only): 1 rows of a real array
    // (read as L complex pairs) -> the L + 1 spectral values of the 2L-point
    // real transform; 2 the inverse (L + 1 values -> 2L reals, kept half
    // written as L complex pairs); 4 fused pass on a half spectrum (the last
    // axis index k3 in [0, N] is not folded).  tw_big: the 2L-point table.
    int real_mode;
    // 1: the table covers every spectral index of the L^d box (no octant
    // fold): flat = k * L^(d-1) + column (convection kernel)
    int table_full;
    // specialised kernels: bit 0 streaming (non-temporal) loads, bit 1
    // streaming stores; allowed when every column tile row starts on a
    // 128-byte line (pitches multiples of 128 bytes) or the pass is a row
    // pass, so that they cover whole lines
    int stream;
};

// Fused 3D column passes whose complex64 kernel stages the Khat tile through
// LDS: the tile width (columns) of the staged kernel, 0 where the entries are
// fetched per thread.  Their plans' FP32 tables (complex ones only at width
// 8) carry the boundary block (PassDesc::tab_bnd) at that stride, so that
// every run they read sits in one line.  Measured faster at 2N = 192, 256, 512 (tiles of 16) and 1024
// (tiles of 8); at 2N = 96 and 128 the table is L2-resident and the staging
// gains nothing.
__host__ __device__ constexpr int staged_fetch_C(int L) {
    return (L == 192 || L == 256 || L == 512) ? 16 : (L == 1024 ? 8 : 0);
}

// Column tile width of the plain forward / inverse complex64 passes of
// length 1024 (16 pencils, 128-byte rows, split exchange); 0: the length's
// default width (8 there).  3D N = 512: those passes 1.39 / 1.34 ms with 8.
__host__ __device__ constexpr int wide_col_C(int L, int mode, int kind, bool fp64) {
    return (L == 1024 && mode == MODE_COL && !fp64 && (kind == KIND_FWD || kind == KIND_INV)) ? 16 : 0;
}

// ----------------------------------------------------- plan precompute ----
struct GreensParams {
    int d;
    int kernel;      // vg_kernel: 0 Laplace, 1 Helmholtz, 2 biharmonic, 3 Delta (Delta + k^2)
    double k, L;
    double ds;       // lattice spacing 2 pi / P
    // 2D Helmholtz constants H_0^(1)(kL), H_1^(1)(kL) and Taylor
    // coefficients of the numerator about s = k.
    double H0r, H0i, H1r, H1i;
    int ntaylor;
    double taylor_r[24], taylor_i[24];
    double window;
    // full-lattice generator (convection kernel): lattice of M points per axis
    // in FFT order, G evaluated at |s_m - h| (with kernel = Helmholtz, k = |h|)
    int full;
    int M;
    double h[3];
};

// Grouped launch of one specialised pass over several arrays: device arrays
// of nitems descriptors and nitems + 1 workgroup offsets (starts[nitems] =
// ntiles, the grid size).
struct GroupArgs {
    const PassDesc* descs;
    const unsigned* starts;
    int nitems;
    unsigned ntiles;
};

// ------------------------------------------------------------- launchers --
// All return hipSuccess or the first HIP error.
hipError_t launch_fft_pass(const PassDesc& p, int mode, int kind, bool fp64, hipStream_t s);
// Grouped specialised pass; `proto` is any of the group's descriptors (the
// launch shape comes from it).  hipErrorInvalidValue if the length has no
// grouped kernel.
hipError_t launch_fast_group(const PassDesc& proto, const GroupArgs& g, int mode, int kind, bool fp64,
                             hipStream_t s);
// Whether launch_fast_group covers passes of length L.
bool fast_group_supported(int L);
size_t fft_pass_lds_bytes(const PassDesc& p, int kind, bool fp64);

hipError_t launch_greens_contract(const GreensParams& g, int M2, int n_out, const double* cmat,
                                  c64* out, hipStream_t s);
hipError_t launch_cos_contract(const c64* in, c64* out, const double* cmat, long long O, int Min,
                               int Nout, long long I, hipStream_t s);
// FP64 octant (rows of N1 entries, dense) -> the kernel table: rows at pitch
// `pitch`, rounded to FP32 (to_fp32) and kept complex or real; with nb > 0
// (3D), entries k3 = bs (b + 1), b < nb, are also written to the boundary
// block at element offset bnd, index (k2 nb + b) N1 + k1.
hipError_t launch_round_table(const c64* in, void* out, long long rows, int N1, int pitch, int to_fp32,
                              int complex_out, long long bnd, int nb, int bs, hipStream_t s);
// First contraction on the full lattice (g.full): rows = M^(d-1), K = M.
hipError_t launch_greens_contract_full(const GreensParams& g, int n_out, const double* cmat, c64* out,
                                       hipStream_t s);
// out[i] = a[i] + sign * i * b[i]
hipError_t launch_combine(const c64* a, const c64* b, c64* out, long long n, int sign, hipStream_t s);

}  // namespace vg
