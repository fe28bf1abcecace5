/* simplexgp.h — C ABI of the MI355X permutohedral-lattice kernel library.
 *
 * The library computes the Simplex-GP kernel operator of Kapoor, Finzi, Wang
 * and Wilson, "SKIing on Simplices: Kernel Interpolation on the
 * Permutohedral Lattice for Scalable Gaussian Processes" (ICML 2021,
 * arXiv:2106.06695):
 *
 *     K ~= W_X K_UU W_X^T      (Section 4, eq. ski_to_bf)
 *
 * where W_X^T is the splat of point values onto the vertices of their
 * enclosing simplices with barycentric weights, K_UU is the blur along the
 * d+1 lattice directions with a stencil sampled from the kernel, and W_X is
 * the slice back to the points (Section 3.2, paragraphs Splat, Blur and
 * Slice), and conjugate-gradient solves with K + noise*I that use only such
 * matrix-vector products (Section 2, Krylov methods).
 *
 * Conventions for every call:
 *   - Array arguments are DEVICE pointers unless marked "host". They are
 *     owned by the caller, dense and row-major (the last index is
 *     contiguous). The library never frees or retains them beyond the call,
 *     except that a lattice keeps its own copies of what it needs (it does
 *     not keep X).
 *   - `stream` is a hipStream_t (NULL = the legacy default stream). Work is
 *     ordered on that stream. lattice_mvm is fully asynchronous; calls that
 *     return host values (lattice_build, cg_solve, lattice_export)
 *     synchronise the stream before returning.
 *   - Every call returns an SGP_* status. On failure sgp_last_error() gives
 *     a message (thread-local; valid until the next failing call on the
 *     same thread). Argument checks run on the host before any GPU work, so
 *     SGP_EINVAL from them leaves the device untouched.
 *   - A lattice handle holds work buffers that lattice_mvm and cg_solve
 *     reuse: calls on ONE handle must not overlap in time (use one stream
 *     per handle, or order them). Different handles are independent.
 */
#ifndef SIMPLEXGP_H
#define SIMPLEXGP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sgp_lattice sgp_lattice; /* opaque; owned by the library */

enum sgp_status {
  SGP_OK = 0,
  SGP_EINVAL = -1,    /* bad argument, or non-finite values in X */
  SGP_ENOMEM = -2,    /* device or host allocation failed */
  SGP_EOVERFLOW = -3, /* a lattice coordinate leaves int32 (|x|/l too large) */
  SGP_EHIP = -4,      /* HIP runtime error */
  SGP_EHASH = -5      /* lattice hash table full at its largest size, or its
                         key check failed for 4 seeds */
};

/* Blur order over the d+1 lattice directions (Section 3.2, Blur). The
 * directions are applied one after another over a fixed point set; on a
 * truncated lattice the result depends on the order:
 *   FORWARD   directions 0, 1, ..., d   (the paper's sequential blur)
 *   REVERSE   directions d, ..., 1, 0   (the transpose of FORWARD)
 *   SYMMETRIC (FORWARD + REVERSE) / 2   (exactly symmetric; default) */
enum sgp_blur { SGP_BLUR_SYMMETRIC = 0, SGP_BLUR_FORWARD = 1, SGP_BLUR_REVERSE = 2 };

/* Stationary kernel whose samples k(t s), t = -r..r, form the blur stencil;
 * the spacing s balances spatial and spectral coverage (Section 4.1,
 * eq. balance_coverage). */
enum sgp_kernel { SGP_KERNEL_RBF = 0, SGP_KERNEL_MATERN32 = 1 };

typedef struct sgp_opts {
  int32_t order;     /* stencil half-width r, 1..8 (default 1, the paper's setting) */
  int32_t kernel;    /* enum sgp_kernel (default SGP_KERNEL_RBF) */
  int32_t blur;      /* enum sgp_blur (default SGP_BLUR_SYMMETRIC) */
  float outputscale; /* sigma_f^2 multiplying the whole operator (default 1) */
  float load_factor; /* hash table fill bound relative to n(d+1), in (0, 0.9]; 0 (default) =
                        automatic: the shape sgp_autotune_build chose for builds of this
                        d and size class, else 0.5 */
  int64_t solve_rows; /* cg_solve uses only the first solve_rows points (0 = all, default):
                         the others splat zero and get x = 0, so a lattice built on
                         [X; X_test] solves with X's block of the joint operator and one
                         lattice_mvm of [x; 0] gives the predictive mean at X_test
                         (Section 2, eq. gp_pred_mean) */
} sgp_opts;

/* Fill *o with the defaults above (host). */
void sgp_opts_default(sgp_opts* o);

/* Build the lattice of the points X (n x d, fp32) with per-dimension
 * lengthscales (host, d doubles, each finite and > 0). Computes the
 * enclosing simplex and barycentric weights of every point (Section 3.2,
 * Splat), inserts every vertex into a GPU hash table, numbers the m
 * distinct lattice points by first occurrence in the (point, vertex) scan,
 * and tabulates the neighbours of each lattice point along each direction
 * (Section 3.2, Blur).
 * Limits: n >= 1, 1 <= d <= 32, n*(d+1) <= 2^30, 0 <= opts->solve_rows <= n.
 * Errors: SGP_EINVAL (arguments, NaN/Inf in X), SGP_EOVERFLOW (|x_j|/l_j so
 * large that a lattice coordinate leaves int32), SGP_ENOMEM, SGP_EHIP,
 * SGP_EHASH. On success *out receives a handle to free with lattice_free.
 * Synchronises `stream` (the lattice size m is read back). */
int lattice_build(const float* X, int64_t n, int32_t d, const double* lengthscales,
                  const sgp_opts* opts /* host; NULL = defaults */, void* stream,
                  sgp_lattice** out);

/* out = outputscale * W_X K_UU W_X^T values, per column (eq. ski_to_bf).
 * values, out: n x C fp32, C >= 1; out must not overlap values.
 * Asynchronous on `stream`. */
int lattice_mvm(const sgp_lattice* L, const float* values, int32_t C, float* out, void* stream);

/* lattice_mvm for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same operation, kernels and results as lattice_mvm, bit for bit, but
 * the MVM's work memory (the lattice values, the splat's partial rows and
 * fragments: 4 (4m + runs) C bytes, runs <= n(d+1)) is one fixed array of
 * SGP_NOALLOC_SCRATCH_BYTES per device, part of the library's code object and
 * held until the process ends. The call makes no device allocation and no
 * allocating library call. The caller still passes values and out (n x C
 * fp32, not overlapping). Every call on one device shares that device's
 * array, and it keeps the last call's contents: calls that overlap in time on
 * one device (different streams or threads) race and give wrong results;
 * order them. The lattice's device must be current.
 * Errors: SGP_EINVAL for NULL or overlapping arrays, C < 1, another device
 * current, or work memory beyond SGP_NOALLOC_SCRATCH_BYTES (the message gives
 * the size needed); SGP_EHIP if the array's device address is unavailable. */
#define SGP_NOALLOC_SCRATCH_BYTES (64ll << 20)
int lattice_mvm_noalloc(const sgp_lattice* L, const float* values, int32_t C, float* out,
                        void* stream);

/* Conjugate gradients on (outputscale*K + noise*I) x = rhs, each of the C
 * columns an independent recurrence from x0 = 0 (Section 2, Krylov methods;
 * Section 5.4 for the tolerance semantics). A column stops when its
 * recursive residual ||r||/||rhs|| <= tol, or after max_iter iterations;
 * tol = 0 runs exactly max_iter iterations. Non-convergence is not an error.
 * Internally the iteration vectors, the lattice values of its MVMs and all
 * reductions are fp64 (the weights stay fp32), so the recursive residual
 * tracks the true residual at tolerances down to ~1e-8 on systems of
 * condition ~1e4; rhs and x are fp32.
 * rhs, x: n x C fp32 device arrays, 1 <= C <= 64, x must not overlap rhs.
 * iters, rel_residual: host arrays of C entries (or NULL) receiving the
 * iterations taken and the final recursive relative residual.
 * noise >= 0, tol >= 0, max_iter >= 1. Synchronises `stream` before it
 * returns (it polls convergence every few iterations). */
int cg_solve(const sgp_lattice* L, const float* rhs, int32_t C, float noise, float tol,
             int32_t max_iter, float* x, int32_t* iters /* host */,
             float* rel_residual /* host */, void* stream);

/* Gradient of L = sum_{i,c} G[i,c] * (outputscale * K V)[i,c] with respect
 * to the points X and the log-lengthscales, by one filtering of the 2(d+1)
 * channels [v, z*v, g, z*g] per column with the kernel derivative
 * k' = dk/d(dist^2), z = x / l (Section 4.2). For the RBF kernel k' = -k/2,
 * so K' is -1/2 times this lattice's operator; other kernels give
 * SGP_EINVAL. The formula assumes a symmetric kernel matrix, so it is the
 * gradient of the SYMMETRIC-order operator's approximation; with FORWARD or
 * REVERSE order the same filtering is applied with that order.
 * X: n x d fp32 device, the points the lattice was built from (same order).
 * V, G: n x C fp32 device. dX: n x d fp32 device output (or NULL).
 * dlogell: host array of d doubles (or NULL). The channels are formed and
 * combined in fp64 and filtered in fp32 (as lattice_mvm), up to 128
 * channels (several columns) at a time, in narrower MVMs on large lattices.
 * Allocates stream-ordered work memory of about 8 n min(128, 2(d+1)C) + 8 n d
 * bytes plus the lattice's fp32 work buffer for one such MVM, and
 * synchronises `stream`. The dV term of the adjoint is K G itself
 * (lattice_mvm). */
int lattice_mvm_grad(const sgp_lattice* L, const float* X, const float* V, const float* G,
                     int32_t C, float* dX, double* dlogell /* host */, void* stream);

/* Sizes of a built lattice (host outputs, any may be NULL): n, d, the
 * number m of lattice points (m <= n(d+1); the lattice-size table of
 * Section 5.2 reports m for the paper's datasets) and the device bytes the
 * handle holds. */
int lattice_info(const sgp_lattice* L, int64_t* n, int32_t* d, int64_t* m,
                 int64_t* device_bytes);

/* Copy the lattice structure to HOST arrays (any may be NULL): the lattice
 * points generated by the splat and the enclosing simplex of every point
 * (Section 3.2, Splat; a vertex k of a point's simplex is its remainder-0
 * lattice point plus the canonical simplex vertex s_k permuted by the ranks
 * of the residuals, eq. canon_simplex), and the blur's neighbour table
 * (Section 3.2, Blur). Lattice points are numbered by first occurrence in
 * the (point, vertex) row-major scan, which makes the export independent of
 * the hash table and of the internal order.
 *   keys m x d      int32  first d coordinates of each lattice point
 *                          (the last is minus their sum)
 *   idx  n x (d+1)  int32  lattice point of vertex k of point i's simplex
 *   w    n x (d+1)  fp32   barycentric weight of that vertex
 *   nbr  m x (d+1) x 2r int32  neighbour of point j along direction k at
 *                          offsets t = -r..-1, 1..r; -1 where absent.
 * Synchronous. */
int lattice_export(const sgp_lattice* L, int32_t* keys, int32_t* idx, float* w, int32_t* nbr);

/* Release a lattice and its device memory (NULL is a no-op). Waits for the
 * device to finish work that may still use it. */
void lattice_free(sgp_lattice* L);

/* Message of the last failure on this thread ("" if none). */
const char* sgp_last_error(void);

/* Device memory from the caller's allocator (process-wide; the interface's
 * handle on memory management, so that the library's buffers come out of,
 * e.g., a framework's caching allocator). alloc(bytes, stream) returns device
 * memory of the current device usable in stream order on `stream` (a
 * hipStream_t), or NULL on failure (the call then fails with SGP_ENOMEM);
 * free(ptr, stream) takes back a block that alloc returned, either after
 * the device has finished every use of it or with `stream` ordering every
 * use, so a stream-ordered allocator may hand it out again to later work on
 * that stream. Lattices, build temporaries and gradient work buffers use it;
 * the library's own idle-block cache is bypassed while it is set. The hooks
 * are called with a library lock held and must not call the library.
 * Both NULL restores the built-in stream-ordered pool; one NULL is
 * SGP_EINVAL. The allocator can change only while the library holds no
 * device block (every lattice freed): otherwise SGP_EINVAL and nothing
 * changes. Returns SGP_OK. */
int sgp_set_allocator(void* (*alloc)(size_t bytes, void* stream), void (*free)(void* ptr, void* stream));

/* The library's idle-block cache on the current device (host outputs, may
 * be NULL): bytes and blocks of device memory freed by lattices and kept for
 * reuse (at most a quarter of the device memory). When an allocation from
 * the built-in pool runs out of memory, the cache is first returned to the
 * pool and the allocation tried once more, so cached blocks never cause
 * SGP_ENOMEM. Returns SGP_OK. */
int sgp_cache_info(int64_t* bytes, int32_t* blocks);

/* Test hook for the out-of-memory path: the next `count` allocations from
 * the built-in pool (on any device) report out-of-memory without asking the
 * device. 0 cancels. Returns SGP_OK. */
int sgp_debug_inject_oom(int32_t count);

/* CG iterations as HIP graphs (process-wide switch, default on). When on,
 * cg_solve records a block of iterations (4 between convergence polls, 8
 * when tol == 0) into a graph once per call and replays it, which removes
 * the per-launch host cost; the arithmetic and results are identical to the
 * launch-by-launch path, which runs when the switch is off, while the
 * profiler is enabled, and for the iterations that do not fill a block.
 * Returns the previous setting. */
int sgp_cg_graph_enable(int on);

/* Fused blur steps (process-wide switch, default on). With a three-tap
 * stencil (order 1), two consecutive direction steps of the blur (Section
 * 3.2, Blur) run as one launch that forms the first step's values at the
 * three neighbours it needs in the same order as a separate step would, so
 * results are bitwise identical with the switch off. Returns the previous
 * setting. */
int sgp_blur_fuse_enable(int on);

/* Sequential chains of the symmetric blur (process-wide). When the four
 * lattice value arrays of an MVM exceed `bytes` in all, the fused launches
 * that advance the forward and the reverse chain separately run one chain
 * after the other (all of one chain's, then the other's) instead of both
 * chains in one launch, so that a launch's arrays share the Infinity Cache.
 * Every row is computed as before, so results are bitwise identical for any
 * setting. bytes < 0: never. The default is SGP_BLUR_SEQ_MIB MiB from the
 * environment, else 128 MiB. Returns the previous threshold. */
int64_t sgp_blur_seq_bytes(int64_t bytes);

/* CG direction update fused into the splat (process-wide switch, default
 * on). Each iteration's x += alpha p and p = r + beta p (Section 2, the
 * conjugate-gradient recurrence) then run in the next iteration's splat,
 * which reads every element of p anyway, and the last one in the final copy
 * of x; off, they run as a pass of their own. The arithmetic is the same, so
 * results are bitwise identical either way. Returns the previous setting. */
int sgp_cg_fuse_enable(int on);

/* Autotuning of the MVM's launch shape (the multi-column lattice filter of
 * Section 3.2, batched as in the mBCG solver of Section 2). Times every
 * candidate on lattice L for C columns, fp64 (the CG path, C <= 64) or
 * fp32 (lattice_mvm), with reps timed MVMs each after one warm-up: the
 * channel chunk width (the widest that fits the LDS budget, half, quarter)
 * times the resident blocks per CU of the persistent splat and slice (as
 * many as fit, or one). The fastest is kept process-wide for lattices of
 * the same d, column width class (C rounded up to a power of two), element
 * size and size class (m rounded up to a power of two) and is used by later
 * lattice_mvm and cg_solve calls; no choice changes any result bit.
 * Allocates two n x C work arrays for the duration of the call and
 * synchronises the stream. choice (may be NULL) receives {chunk width,
 * splat blocks per CU, slice blocks per CU} (0: as many as fit);
 * ms_per_mvm (may be NULL) the fastest time. Returns SGP_EINVAL for a NULL
 * lattice, C < 1, C > 64 in fp64 or reps < 1. */
int sgp_autotune(const sgp_lattice* L, int32_t C, int32_t fp64, int32_t reps, void* stream,
                 int32_t* choice, float* ms_per_mvm);

/* Forget every autotuned choice, the MVM's and the build's (later calls use
 * the default shapes). */
int sgp_autotune_reset(void);

/* Autotuning of the lattice build's hash table (the table into which every
 * simplex vertex is inserted, Section 3.2, Splat): times lattice_build of X
 * (reps timed builds after one warm-up, each synchronised and freed) for
 * each candidate table shape, i.e. a load factor (full table of
 * n(d+1)/load_factor slots) and the first attempt's reduction of it by
 * 2^shrink (a build whose reduced table fills up repeats with the full one),
 * and keeps the fastest process-wide for builds of the same d and size class
 * (n(d+1) rounded up to a power of two) whose opts->load_factor is 0. No
 * choice changes any result: lattice points are numbered by first
 * occurrence, not by table slot. opts as for lattice_build (its load_factor
 * is ignored). Outputs (host, may be NULL): the chosen load factor and
 * shrink, and the time of one build with them. Errors as lattice_build,
 * and SGP_EINVAL for reps < 1. Synchronises `stream`. */
int sgp_autotune_build(const float* X, int64_t n, int32_t d, const double* lengthscales,
                       const sgp_opts* opts, int32_t reps, void* stream, float* load_factor,
                       int32_t* shrink, float* ms_per_build);

/* Kernel timing with HIP events, for benchmarks. While enabled, every
 * kernel launch of the library is bracketed by two events on its stream.
 * sgp_profile_read synchronises the recorded events and reports, for one
 * kernel kind, the number of launches and their summed duration in ms
 * since the last reset. Kinds are numbered 0..sgp_profile_kinds()-1. */
int sgp_profile_enable(int on);
int sgp_profile_reset(void);
int sgp_profile_kinds(void);
const char* sgp_profile_name(int kind);
int sgp_profile_read(int kind, int64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif
#endif /* SIMPLEXGP_H */
