/* Simplex-GP lattice oracle: plain, single-threaded, fp64 CPU implementation.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library includes,
 * links or calls this code; it exists so that tests, the smoke check and the
 * benchmark's CPU-baseline leg can compare the GPU path against an
 * implementation written directly from the paper (Kapoor et al., "SKIing on
 * Simplices", ICML 2021, arXiv:2106.06695):
 *
 *   - permutohedral lattice and canonical simplex ........ Section 3.2, eq. canon_simplex
 *   - splat: elevation, enclosing simplex, barycentric ... Section 3.2, paragraph "Splat"
 *   - blur along the d+1 lattice directions .............. Section 3.2, paragraph "Blur"
 *   - slice with the cached weights ...................... Section 3.2, paragraph "Slice"
 *   - K ~ W K_UU W^T (splat, blur, slice) ................ Section 4, eq. ski_to_bf
 *   - stencil k(i s), i = -r..r, spacing from coverage ... Section 4.1, eq. balance_coverage
 *   - conjugate gradients with MVMs only ................. Section 2 (Krylov methods), Section 5.4
 *   - MVM gradient via k' filtering ...................... Section 4.2
 *
 * Every array is host memory, row-major. Return codes: 0 ok, -1 bad argument,
 * -3 overflow of the int32 key range.
 */
#ifndef SGP_ORACLE_H
#define SGP_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_KERNEL_RBF = 0, ORC_KERNEL_MATERN32 = 1 };
enum { ORC_BLUR_SYMMETRIC = 0, ORC_BLUR_FORWARD = 1, ORC_BLUR_REVERSE = 2 };

/* Spacing s, stencil w[0..2r] (= k(t s) for t=-r..r), elevation scale alpha
 * and per-dimension factors f[0..d-1]. */
int orc_constants(int d, int r, int kernel, const double* ell, double* s,
                  double* stencil, double* alpha, double* f);

/* Elevated points y (n x (d+1)). */
int orc_embed(const float* X, int64_t n, int d, const double* ell, int r, int kernel,
              double* y);

/* Enclosing simplex per point: keys (n x (d+1) x d, vertex k's stored
 * coordinates), barycentric weights (n x (d+1)), remainder-0 point and rank
 * after the sum fix (n x (d+1) each). Any output may be NULL. */
int orc_simplex(const float* X, int64_t n, int d, const double* ell, int r, int kernel,
                int32_t* keys, double* bary, int32_t* r0, int32_t* rank);

/* Whole lattice (splat structure + neighbour table). NULL on error. */
void* orc_build(const float* X, int64_t n, int d, const double* ell, int r, int kernel);
int64_t orc_num_vertices(const void* lat);
/* keys m x d, idx n x (d+1), w n x (d+1), nbr m x (d+1) x 2r with the 2r
 * offsets ordered t = -r..-1, 1..r. Any output may be NULL. */
int orc_export(const void* lat, int32_t* keys, int32_t* idx, double* w, int32_t* nbr);
void orc_free(void* lat);

/* out = outputscale * W B W^T V for the chosen blur order (n x C). */
int orc_mvm(const void* lat, const double* V, int C, int mode, double outputscale,
            double* out);
/* out = W^T V (m x C) and out = W U (n x C): the two halves of the MVM. */
int orc_splat(const void* lat, const double* V, int C, double* U);
int orc_slice(const void* lat, const double* U, int C, double* out);
/* One blur pass over lattice values U (m x C) in place. */
int orc_blur(const void* lat, double* U, int C, int mode);

/* CG on A = outputscale*K_lat + noise*I, each of the C columns separately,
 * x0 = 0. Stops a column when ||r||/||b|| <= tol (recursive residual) or at
 * max_iter. iters[c], rel_rec[c] (recursive) and rel_true[c] (from a fresh
 * MVM) are written per column; any of them may be NULL. */
int orc_cg(const void* lat, const double* B, int C, int mode, double outputscale,
           double noise, double tol, int max_iter, double* X, int32_t* iters,
           double* rel_rec, double* rel_true);
/* The same restricted to the first `rows` points (rows <= 0: all): the other
 * points splat zero, are not solved for, and get x = 0. B and X stay n x C. */
int orc_cg_rows(const void* lat, const double* B, int C, int mode, double outputscale,
                double noise, double tol, int max_iter, int64_t rows, double* X,
                int32_t* iters, double* rel_rec, double* rel_true);

/* Gradient of L = sum_{i,c} G[i,c] * (K_lat V)[i,c] (outputscale 1) with
 * respect to the inputs X (n x d) and the log-lengthscales (d), from one k'
 * filtering of the concatenated channels of Section 4.2. */
int orc_mvm_grad(const float* X, int64_t n, int d, const double* ell, int r, int kernel,
                 int mode, const double* V, const double* G, int C, double* dX,
                 double* dlogell);

#ifdef __cplusplus
}
#endif
#endif
