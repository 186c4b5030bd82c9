/*
 * vg.h -- C ABI of the MI355X (gfx950) volume-potential library.
 *
 * The library computes the volume potential of the Introduction of Vico,
 * Greengard and Ferrando, "Fast convolution with free-space Green's functions":
 *
 *     phi(x) = int_D g_k(x - y) f(y) dy,     D = [-1/2, 1/2]^d,  d in {2, 3},
 *
 * with g_k the free-space Laplace kernel (k = 0: 1/(4 pi r) in 3D,
 * -(1/2 pi) log r in 2D) or Helmholtz kernel (e^{ikr}/(4 pi r) in 3D,
 * (i/4) H_0^(1)(k r) in 2D, Table 2), by the truncated-kernel method:
 *   - plan time (Sections 2 and 4): the Fourier transform of the kernel
 *     truncated at radius L (Tables 1 and 2) is sampled in FP64 on the
 *     P N-per-axis lattice, inverse transformed into the discrete operator T
 *     (the response to a unit density at one grid point), and T is transformed
 *     over the (2N)^d box into the table Khat used by every apply;
 *   - apply time (Section 4): phi_{i'} = sum_i T(i' - i) f_i, evaluated as
 *     zero padding to (2N)^d, forward FFT, multiplication by Khat, inverse FFT
 *     and cropping, in hand-written HIP kernels;
 *   - gradient (abstract, Section 3): one more inverse FFT per component after
 *     multiplying the spectrum by i kappa_j.
 *
 * Grid and layout (Section 4).  h = 1/N with N even; along every axis array
 * index a in [0, N) is the point x_a = (a - N/2 + 1) h.  Densities and
 * potentials are dense C-ordered arrays of N^d interleaved complex numbers
 * (x_1 slowest, x_d fastest): float2 {re, im} for FP32 plans, double2 for FP64
 * plans.  phi_{i'} = sum_i T(i' - i) f_i already carries the quadrature weight
 * h^d.  The sign convention is phi = g * f, i.e. (Delta + k^2) phi = -f.
 *
 * Memory.  Every array argument of the apply calls is a DEVICE pointer on the
 * current HIP device and is owned by the caller; the library owns its plan
 * tables.  `stream` is a hipStream_t passed as void* (NULL = the null stream).
 * Apply calls are asynchronous on `stream`; faults inside kernels surface at the
 * caller's next synchronisation.  Plans are immutable after creation and may be
 * used from several threads, except that calls passing workspace == NULL share
 * the plan's internal workspace and must not overlap in time.
 *
 * Errors.  Every call returns a vg_status; no C++ exception crosses the ABI.
 * vg_last_error() returns a thread-local message describing the last failure on
 * the calling thread.
 */
#ifndef VG_H
#define VG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum vg_status {
    VG_OK = 0,
    VG_ERR_INVALID_ARG = 1,      /* bad dimension, size, kernel, k, pointer, option */
    VG_ERR_UNSUPPORTED_SIZE = 2, /* 2N has a prime factor above 7, or exceeds a limit */
    VG_ERR_OUT_OF_MEMORY = 3,    /* device or host allocation failed */
    VG_ERR_NO_DEVICE = 4,        /* no HIP device is visible */
    VG_ERR_DEVICE = 5,           /* a HIP runtime call or kernel launch failed */
    VG_ERR_NOT_CAPTURABLE = 6,   /* the call cannot run inside stream capture */
    VG_ERR_INTERNAL = 7          /* a bug: please report */
} vg_status;

/* The kernels of Tables 1 (3D) and 2 (2D), with the tables' Green's functions
 * (each satisfies L g = -delta for its operator L, except Delta(Delta + k^2),
 * whose tabulated g_k - g_0 satisfies Delta(Delta + k^2) g = k^2 delta). */
typedef enum vg_kernel {
    VG_LAPLACE = 0,           /* Delta:        1/(4 pi r) (3D),  -(1/2 pi) log r (2D) */
    VG_HELMHOLTZ = 1,         /* Delta + k^2:  e^{ikr}/(4 pi r) (3D), (i/4) H_0^(1)(kr) (2D) */
    VG_BIHARMONIC = 2,        /* Delta^2:      r/(8 pi) (3D), -(r^2/(8 pi))(log r - 1) (2D) */
    VG_LAPLACE_HELMHOLTZ = 3, /* Delta (Delta + k^2): g_k - g_0, the difference of the two above */
    VG_CONVECTION = 4         /* Delta - 2i h.grad (vector h = opts.h, |h| > 0): e^{i h.x} g_{|h|}(x);
                               * truncated transform G^L_{|h|}(|s - h|), not radial (Tables 1-2) */
} vg_kernel;

typedef enum vg_precision {
    VG_FP32 = 0,  /* complex64 densities and FFTs; tables built in FP64, rounded once */
    VG_FP64 = 1   /* complex128 end to end */
} vg_precision;

/* Plan-time autotuning: the apply program is timed (on zero arrays, on the
 * plan's stream, synchronously) under candidate layouts and the fastest is
 * kept for apply and gradient.  Candidates: the plan's default layout, pitch
 * padding of the 2N x 2N planes (3D) / 2N rows (2D) of the intermediates,
 * XCD-aware tile order of the specialised kernels, the four-step split
 * 2N = L1 L2 of long 2D columns, and (full) every pass on the generic
 * runtime-radix kernel.
 * The choice is persisted in a JSON file ($VG_TUNE_CACHE; empty disables it;
 * default $XDG_CACHE_HOME/vgconv/tune.json or ~/.cache/vgconv/tune.json)
 * under a key of (d, N, table class, precision, tune mode, device
 * architecture and compute units, library build); a later plan with the same
 * key takes the stored layout without timing.  A missing, corrupt or stale
 * file means tuning as without a cache; a file that cannot be written is
 * ignored. */
typedef enum vg_tune_mode {
    VG_TUNE_OFF = 0,    /* built-in layout: 256-byte padding, XCD order, default split */
    VG_TUNE_QUICK = 1,  /* padding {256, 0} x order {XCD, launch} (x 3 splits in 2D), 3 timed applies each */
    VG_TUNE_FULL = 2    /* padding {0, 256, 512, 1024} x order x 6 splits, plus generic kernels, 10 applies each */
} vg_tune_mode;

typedef struct vg_plan vg_plan;

/* Plan options (vg_plan_create_ex).  Zero-initialised fields take defaults. */
typedef struct vg_plan_opts {
    int precision;       /* vg_precision, default VG_FP32 */
    double L;            /* truncation radius, must exceed sqrt(d); 0 -> 1.8 (3D), 1.5 (2D) (Section 2) */
    int P;               /* precompute oversampling, must satisfy P > 1 + L; 0 -> 4 (Section 2) */
    int tune;            /* vg_tune_mode, default VG_TUNE_OFF */
    int keep_operator;   /* nonzero: keep T (FP64) on the device for vg_plan_operator_entries */
    void* stream;        /* hipStream_t for the precompute, NULL = null stream */
    double h[3];         /* VG_CONVECTION: the vector h (h[2] unused in 2D); ignored by the other kernels */
} vg_plan_opts;

/* Plan description returned by vg_plan_get_info. */
typedef struct vg_plan_info {
    int d, N;
    int kernel;          /* vg_kernel */
    int precision;       /* vg_precision */
    double k, L;
    int P;
    double precompute_ms;     /* device time of the FP64 precompute (kernel spectrum -> T -> Khat) */
    size_t table_bytes;       /* device bytes of the kernel table kept for applies: the Khat octant
                                 ((N+1)^d entries; 3D rows padded to 16 entries from N = 96 on;
                                 FP32 3D N = 96, 128, 256 add a block repeating every 16th k3
                                 entry, complex N = 512 every 8th) or, for the convection
                                 kernel, the full (2N)^d table */
    size_t workspace_bytes;   /* vg_workspace_size */
    size_t gradient_workspace_bytes;
    int tune;                 /* vg_tune_mode the plan was created with */
    double tune_ms;           /* host wall time of the autotuner (0 without tuning) */
    int tune_candidates;      /* layouts timed */
    int pad_bytes;            /* chosen layout: pitch padding of the intermediates */
    int xcd_map;              /* 1: XCD-aware tile order */
    int four_step_L1;         /* four-step split of long 2D columns (0: default / none) */
    int generic_passes;       /* 1: all passes on the generic kernel */
    int tune_cached;          /* 1: the layout was read from the persistent tune cache (no timing) */
} vg_plan_info;

/*
 * Create a plan for d in {2, 3}, even N >= 4 and a vg_kernel.  VG_HELMHOLTZ
 * and VG_LAPLACE_HELMHOLTZ need a finite k > 0 (the others ignore k).
 * VG_CONVECTION needs opts with a finite h of |h| > 0 and ignores k (the
 * plan's k is |h|); its kernel is not symmetric per axis, so the plan keeps
 * the whole (2N)^d spectrum (complex, at most 4 GiB) instead of an octant,
 * and its precompute takes full-lattice sums ((P N)^d evaluations of the
 * transform); 3D plans of it are limited to N <= 256.
 * Runs the FP64 precompute of Sections 2 and 4 on the current device and
 * synchronises before returning.
 * Errors: VG_ERR_INVALID_ARG (bad arguments; *out untouched),
 * VG_ERR_UNSUPPORTED_SIZE (2N has a prime factor above 7, or a pass whose
 * pencil fits no kernel: a 2D row of 2N values must fit one workgroup's LDS,
 * which allows 2N up to 12800 for the lengths with specialised row kernels
 * (complex64; 8192 for complex128) and up to 10240 otherwise),
 * VG_ERR_NO_DEVICE, VG_ERR_OUT_OF_MEMORY, VG_ERR_DEVICE.  On error *out is
 * set to NULL.
 */
vg_status vg_plan_create(int d, int N, vg_kernel kernel, double k, vg_plan** out);
vg_status vg_plan_create_ex(int d, int N, vg_kernel kernel, double k,
                            const vg_plan_opts* opts, vg_plan** out);

/* Release a plan and everything it owns.  NULL is a no-op.  The caller must
 * ensure no apply using the plan is still running. */
void vg_plan_destroy(vg_plan* plan);

/* Fill *info.  Errors: VG_ERR_INVALID_ARG for NULL arguments. */
vg_status vg_plan_get_info(const vg_plan* plan, vg_plan_info* info);

/* Bytes of device workspace an apply / gradient call needs when it is given an
 * explicit workspace (0 for a NULL plan). */
size_t vg_workspace_size(const vg_plan* plan);
size_t vg_gradient_workspace_size(const vg_plan* plan);

/*
 * phi = T * f on the N^d grid (Section 4's discrete convolution).
 * f, phi: device arrays of N^d complex (float2 / double2 per the plan);
 * phi == f (in place) is allowed.  workspace: device buffer of at least
 * vg_workspace_size(plan) bytes, 256-byte aligned, or NULL to use the plan's
 * internal workspace.  Asynchronous on `stream`.
 * Errors: VG_ERR_INVALID_ARG (NULL plan/pointers), VG_ERR_DEVICE (launch).
 */
vg_status vg_apply(const vg_plan* plan, const void* f, void* phi,
                   void* workspace, void* stream);

/*
 * Spectral gradient of phi (abstract and Section 3: one extra inverse FFT per
 * component).  grad: device array of d * N^d complex, component-major
 * (d/dx_1 first), derivatives with respect to the physical coordinates x_j.
 * phi may be NULL; when given it receives the same result as vg_apply.
 * workspace: at least vg_gradient_workspace_size(plan) bytes, or NULL.
 * The derivative multiplies the (2N)^d spectrum by i pi m_j (m_j the signed
 * frequency, zero at the Nyquist index m_j = N).
 * Errors: VG_ERR_INVALID_ARG (NULL plan/f/grad), VG_ERR_UNSUPPORTED_SIZE
 * (2D plans whose two-output gradient rows do not fit in LDS, e.g. 2N =
 * 10240 on the generic kernel; their applies still run), VG_ERR_DEVICE
 * (launch).
 */
vg_status vg_gradient(const vg_plan* plan, const void* f, void* phi, void* grad,
                      void* workspace, void* stream);

/*
 * Real densities: phi = T * f for real f and
 * a real kernel (VG_LAPLACE, VG_BIHARMONIC), where T is real (Sections 2 and
 * 4) and so is phi.  f, phi: device arrays of N^d float (double for FP64
 * plans), C order, the grid of vg_apply; f == phi allowed.  The transforms
 * run on the half spectrum of the last axis (N + 1 of 2N values; a real row
 * is processed as N/2 complex pairs), moving about half the bytes of
 * vg_apply.  workspace: vg_real_workspace_size(plan) bytes, or NULL.
 * Asynchronous on `stream`.
 * Errors: VG_ERR_INVALID_ARG (NULL arguments, complex kernel),
 * VG_ERR_UNSUPPORTED_SIZE (no length-specialised kernels for N or 2N),
 * VG_ERR_DEVICE.
 */
size_t vg_real_workspace_size(const vg_plan* plan);
vg_status vg_apply_real(const vg_plan* plan, const void* f, void* phi, void* workspace, void* stream);

/*
 * Allocation-free apply, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Computes exactly what vg_apply computes (the same kernels and
 * launches; results are bit-identical), with its workspace in a device array
 * owned by the library: VG_NOALLOC_WORKSPACE_BYTES (128 MiB) per GPU, held
 * from library load until the process ends.  The call allocates nothing; the
 * array's device address is looked up once per device, on the first call
 * made with that device current.  The caller passes f and phi as for
 * vg_apply (device arrays of N^d complex; phi == f allowed).
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind: calls that overlap in time on one GPU (different streams or host
 * threads) race and give wrong results.  No pass reads workspace it has not
 * written in the same call, so nothing needs clearing between calls.
 * Errors: VG_ERR_INVALID_ARG (NULL arguments, a plan of another device),
 * VG_ERR_UNSUPPORTED_SIZE (vg_workspace_size(plan) above
 * VG_NOALLOC_WORKSPACE_BYTES: e.g. 3D N > 128 in FP32, N > 96 in FP64),
 * VG_ERR_DEVICE (symbol lookup, launch).
 */
#define VG_NOALLOC_WORKSPACE_BYTES (128u << 20)
vg_status vg_apply_noalloc(const vg_plan* plan, const void* f, void* phi, void* stream);

/*
 * Apply `count` plans to `count` densities in one go: phi[i] = T_i * f[i]
 * (Section 4 applied to a set of independent densities).  Plans may mix d, N,
 * kernel and k; all must share one precision and live on the current device.
 * f[i], phi[i]: device arrays as in vg_apply (phi[i] == f[i] allowed).
 * Execution: stage s runs pass s of every density; densities whose pass s
 * has the same specialised kernel share one grouped launch whose workgroups
 * take (density, tile) items.  The launch sequence is captured in a HIP graph
 * on the first call with a given (plans, f, phi, workspace) and replayed on
 * later calls with the same arguments (the library keeps the last 8 such
 * batches; destroying a plan drops the batches that use it).
 * The call may itself be recorded into the caller's stream capture once the
 * same arguments have been used in one call outside capture.  The recorded
 * launches point into device memory the library keeps for that batch (its
 * descriptors and, with workspace == NULL, the internal workspace): such a
 * batch is never evicted from the cache and keeps that memory until one of
 * its plans is destroyed, after which the caller's graph must not be
 * launched again.
 * workspace: at least vg_batched_workspace_size bytes, or NULL (an internal
 * buffer owned by the library; such calls must not overlap in time).
 * Errors: VG_ERR_INVALID_ARG (count <= 0, NULL entries, mixed precision, a
 * plan of another device), VG_ERR_NOT_CAPTURABLE (first use of these
 * arguments, or growth of the internal workspace, under stream capture),
 * VG_ERR_OUT_OF_MEMORY, VG_ERR_DEVICE.
 */
size_t vg_batched_workspace_size(int count, const vg_plan* const* plans);
vg_status vg_apply_batched(int count, const vg_plan* const* plans,
                           const void* const* f, void* const* phi,
                           void* workspace, void* stream);

/*
 * Lippmann-Schwinger solve (Section 5.3, the dual form of the equation): find
 * the density sigma of the scattered field phi_s = g_k * sigma from
 *     -sigma + k^2 q (g_k * sigma) = -k^2 q phi_in
 * by Bi-CGStab (Section 5.3's iteration) started from sigma = 0, with the
 * plan's convolution as the matrix-vector product (two per iteration).
 * plan: a VG_HELMHOLTZ plan (k is the plan's wavenumber).
 * q, phi_in: device arrays of N^d complex (the plan's precision), the
 *   contrast (compactly supported inside the box) and the incident field on
 *   the grid; sigma: device array of N^d complex, the solution.
 * tol: stop when the residual 2-norm is at most tol times that of the
 *   right-hand side; max_iter >= 1 iterations at most.
 * workspace: vg_ls_workspace_size(plan) bytes, or NULL (allocated and freed
 *   inside the call).
 * Synchronous: the call waits on `stream` once per dot product and returns
 * when the iteration stops.  result (may be NULL): iterations, matrix-vector
 * products, final relative residual (of the recurrence), converged flag; not
 * converging within max_iter (or a Bi-CGStab breakdown) is reported there,
 * with status VG_OK.
 * Errors: VG_ERR_INVALID_ARG (NULL arrays, not a Helmholtz plan, tol <= 0,
 * max_iter < 1), VG_ERR_OUT_OF_MEMORY, VG_ERR_DEVICE.
 */
typedef struct vg_ls_result {
    int iterations;
    int matvecs;
    double residual;
    int converged;
} vg_ls_result;

size_t vg_ls_workspace_size(const vg_plan* plan);
vg_status vg_ls_solve(const vg_plan* plan, const void* q, const void* phi_in, void* sigma,
                      double tol, int max_iter, void* workspace, void* stream,
                      vg_ls_result* result);

/*
 * Copy plan tables to host memory, converted to complex128 (interleaved
 * doubles).  Synchronous.
 *   vg_plan_kernel_hat: Khat(m) on the octant m in [0, N]^d, (N+1)^d values,
 *     C order: the spectrum of T on the (2N)^d box (Khat(m) = Khat(2N - m)
 *     per axis), as stored for applies (FP32 plans: rounded to float).
 *     VG_CONVECTION: all of m in [0, 2N)^d, (2N)^d values.
 *   vg_plan_operator_entries: T(n) on n in [0, N)^d, N^d values (T(n) = T(|n|)
 *     per axis); the entries of the high-order Nystrom matrix (Section 4
 *     remark).  VG_CONVECTION: n in [-(N-1), N-1]^d, (2N-1)^d values, C order
 *     of n + N - 1.  Needs opts.keep_operator; VG_ERR_INVALID_ARG otherwise.
 * host_out must hold the stated number of complex128 values.
 */
vg_status vg_plan_kernel_hat(const vg_plan* plan, double* host_out);
vg_status vg_plan_operator_entries(const vg_plan* plan, double* host_out);

/*
 * Pass profiler (diagnostics).  vg_profiler_enable(1): every apply / gradient
 * call records a HIP event between consecutive passes on its stream;
 * vg_profiler_enable(2): only just before and after the call's pass with the
 * most algorithmic bytes (two events per call, so the other passes run as
 * without the profiler); 0 switches it off (other values:
 * VG_ERR_INVALID_ARG).  collect() waits for the recorded events and returns,
 * per pass name, the number of launches and their summed device time, then
 * clears the record.  Each event record adds a few microseconds to the
 * stream.  Process-wide; thread-safe.
 */
typedef struct vg_pass_time {
    char name[32];
    int launches;
    double total_ms;
    double bytes_per_launch;  /* algorithmic HBM bytes of one launch (reads + writes) */
} vg_pass_time;
vg_status vg_profiler_enable(int enable);
vg_status vg_profiler_collect(vg_pass_time* out, int max_entries, int* n_entries);

/*
 * Plain streaming copy of `bytes` bytes (multiple of 16) between device
 * buffers on `stream`: the reference kernel for attainable HBM bandwidth and
 * for calibrating hardware byte counters.  Errors: VG_ERR_INVALID_ARG.
 */
vg_status vg_hbm_copy(void* dst, const void* src, size_t bytes, void* stream);

/* Human-readable name of a status code (never NULL). */
const char* vg_status_string(vg_status status);

/* Message of the last failure on the calling thread ("" if none). */
const char* vg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* VG_H */
