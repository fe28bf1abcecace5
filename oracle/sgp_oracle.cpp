// Simplex-GP lattice oracle (test infrastructure only; see sgp_oracle.h).
//
// Plain single-threaded fp64 code, written for reading against the paper
// rather than for speed: std::unordered_map for the lattice hash table, one
// loop per mathematical sum, no blocking or fusion. Build with
// -ffp-contract=off so that each operation below rounds exactly once.
//
// Readings taken where the paper is silent (each also listed in the design
// notes of the repository):
//   * Scaling: one lattice step along any direction equals s lengthscale
//     units, i.e. the elevation multiplies by alpha = sqrt(d(d+1))/s.
//   * Stencil: unnormalised kernel samples k(|t| s), t = -r..r, so w_0 = 1.
//   * Every vertex of every enclosing simplex is a lattice point, even when
//     its barycentric weight is zero.
//   * Lattice points are numbered by first occurrence in the (point, vertex)
//     row-major scan.
//   * Blur directions are applied one after another, each as a Jacobi update
//     over the fixed point set; a missing neighbour contributes zero.
//     FORWARD runs directions 0..d, REVERSE d..0 and SYMMETRIC averages the
//     two (the truncated forward chain alone is not symmetric).
//   * Rounding to the nearest remainder-0 point uses round-half-to-even and
//     ranks break ties towards the lower coordinate index.
#include "sgp_oracle.h"

#include <cmath>
#include <cstdint>
#include <cstring>
#include <unordered_map>
#include <vector>

namespace {

const double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// Stencil and spacing (Section 4.1, eq. balance_coverage).
// The spatial coverage of m = 2r+1 samples spaced s apart is the kernel mass
// on [-s m/2, s m/2]; the spectral coverage is the mass of its Fourier
// transform below the Nyquist frequency pi/s. Both are written here as
// closed-form fractions for the two kernels supported.

double kernel_value(int kernel, double tau) {
  tau = std::fabs(tau);
  if (kernel == ORC_KERNEL_RBF) return std::exp(-0.5 * tau * tau);
  const double l3 = std::sqrt(3.0);  // Matern nu = 3/2, unit lengthscale
  return (1.0 + l3 * tau) * std::exp(-l3 * tau);
}

// Fraction of the kernel's integral inside [-a, a].
double spatial_coverage(int kernel, double a) {
  if (kernel == ORC_KERNEL_RBF) return std::erf(a / std::sqrt(2.0));
  const double l3 = std::sqrt(3.0);
  // integral_0^a (1 + l3 t) e^{-l3 t} dt = 2/l3 - e^{-l3 a} (2/l3 + a), total 2/l3
  return 1.0 - std::exp(-l3 * a) * (1.0 + l3 * a / 2.0);
}

// Fraction of the Fourier transform's integral inside [-b, b].
double spectral_coverage(int kernel, double b) {
  if (kernel == ORC_KERNEL_RBF) return std::erf(b / std::sqrt(2.0));  // F ~ e^{-w^2/2}
  // F ~ (3 + w^2)^-2; substitute w = sqrt(3) tan(theta)
  const double th = std::atan(b / std::sqrt(3.0));
  return (th + 0.5 * std::sin(2.0 * th)) / (kPi / 2.0);
}

// Spacing s where spatial coverage (increasing in s) meets spectral coverage
// (decreasing in s). The RBF root has the closed form sqrt(2 pi / m).
double spacing(int kernel, int r) {
  const int m = 2 * r + 1;
  if (kernel == ORC_KERNEL_RBF) return std::sqrt(2.0 * kPi / (double)m);
  double lo = 1e-3, hi = 1e3;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    const double gap = spatial_coverage(kernel, mid * m / 2.0) - spectral_coverage(kernel, kPi / mid);
    if (gap < 0.0) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

struct Consts {
  int d = 0, r = 0, kernel = 0;
  double s = 0, alpha = 0;
  std::vector<double> stencil;  // k(t s), t = -r..r
  std::vector<double> f;        // f[j-1] for elevation column j = 1..d
};

int make_consts(int d, int r, int kernel, const double* ell, Consts& c) {
  if (d < 1 || d > 32 || r < 1 || r > 8 || !ell) return -1;
  if (kernel != ORC_KERNEL_RBF && kernel != ORC_KERNEL_MATERN32) return -1;
  for (int j = 0; j < d; ++j)
    if (!(ell[j] > 0.0) || !std::isfinite(ell[j])) return -1;
  c.d = d; c.r = r; c.kernel = kernel;
  c.s = spacing(kernel, r);
  c.stencil.resize(2 * r + 1);
  for (int t = -r; t <= r; ++t) c.stencil[t + r] = kernel_value(kernel, t * c.s);
  c.alpha = std::sqrt((double)(d * (d + 1))) / c.s;
  c.f.resize(d);
  for (int j = 1; j <= d; ++j)
    c.f[j - 1] = c.alpha / (ell[j - 1] * std::sqrt((double)(j * (j + 1))));
  return 0;
}

// ---------------------------------------------------------------------------
// Splat, step 1: elevation into the hyperplane H_d = {y : sum y = 0} with the
// triangular basis whose column j (j = 1..d) is (1,..,1 [j times], -j, 0,..)
// normalised by sqrt(j(j+1)), times alpha / l_j.
void elevate(const float* x, const Consts& c, double* y) {
  const int d = c.d;
  double S = 0.0;
  for (int j = d; j >= 1; --j) {
    const double cj = (double)x[j - 1] * c.f[j - 1];
    y[j] = S - (double)j * cj;
    S = S + cj;
  }
  y[0] = S;
}

const double kKeyLimit = 1073741824.0;  // |y_i| bound that keeps keys in int32

// Splat, step 2: the enclosing simplex (nearest remainder-0 point, ranking of
// the residuals, sum fix) and the barycentric weights.
// Returns 0, -1 on non-finite input, -3 when keys would leave int32.
int enclose(const double* y, int d, int64_t* r0, int* rank, double* bary) {
  const int D = d + 1;
  int64_t delta_sum = 0;
  for (int i = 0; i < D; ++i) {
    if (!std::isfinite(y[i])) return -1;
    if (!(std::fabs(y[i]) <= kKeyLimit)) return -3;
    const double q = std::rint(y[i] / (double)D);  // nearest multiple of d+1
    r0[i] = (int64_t)q * D;
    delta_sum += (int64_t)q;
  }
  std::vector<double> del(D);
  for (int i = 0; i < D; ++i) del[i] = y[i] - (double)r0[i];
  // rank 0 = largest residual; equal residuals go to the lower index first
  for (int i = 0; i < D; ++i) {
    int rk = 0;
    for (int j = 0; j < D; ++j)
      if (del[j] > del[i] || (del[j] == del[i] && j < i)) ++rk;
    rank[i] = rk;
  }
  // The coordinates of the remainder-0 point must sum to zero: move the
  // delta_sum most over-rounded (or under-rounded) coordinates by d+1.
  if (delta_sum > 0) {
    for (int i = 0; i < D; ++i) {
      if (rank[i] >= D - delta_sum) { r0[i] -= D; rank[i] += (int)delta_sum - D; }
      else rank[i] += (int)delta_sum;
    }
  } else if (delta_sum < 0) {
    for (int i = 0; i < D; ++i) {
      if (rank[i] < -delta_sum) { r0[i] += D; rank[i] += (int)delta_sum + D; }
      else rank[i] += (int)delta_sum;
    }
  }
  for (int i = 0; i < D; ++i) del[i] = y[i] - (double)r0[i];
  // Residuals in rank order, each divided by d+1.
  std::vector<double> q(D);
  for (int i = 0; i < D; ++i) q[rank[i]] = del[i] / (double)D;
  // Weight of vertex k is the gap between consecutive sorted residuals
  // (vertex k sits at r0 + the canonical simplex vertex s_k, permuted by rank).
  for (int k = 1; k <= d; ++k) bary[k] = q[d - k] - q[d + 1 - k];
  bary[0] = q[d] + (1.0 - q[0]);
  return 0;
}

// Stored coordinates (the first d of d+1) of vertex k: r0 + s_k permuted by
// rank, where s_k has entries k (for the d+1-k largest residuals) and
// k-(d+1) (for the k smallest), eq. canon_simplex.
void vertex_key(const int64_t* r0, const int* rank, int d, int k, int32_t* key) {
  for (int i = 0; i < d; ++i) {
    int64_t v = r0[i] + k;
    if (rank[i] > d - k) v -= d + 1;
    key[i] = (int32_t)v;
  }
}

struct KeyHash {
  size_t operator()(const std::vector<int32_t>& k) const {
    uint64_t h = 1469598103934665603ull;
    for (int32_t v : k) { h ^= (uint32_t)v; h *= 1099511628211ull; }
    return (size_t)h;
  }
};

struct Lattice {
  int64_t n = 0;
  Consts c;
  int64_t m = 0;
  std::vector<int32_t> idx;   // n x (d+1)
  std::vector<double> w;      // n x (d+1)
  std::vector<int32_t> keys;  // m x d
  std::vector<int32_t> nbr;   // m x (d+1) x 2r
};

int build_lattice(const float* X, int64_t n, const Consts& c, Lattice& L) {
  const int d = c.d, D = d + 1, r = c.r;
  L.n = n; L.c = c; L.m = 0;
  L.idx.assign((size_t)n * D, -1);
  L.w.assign((size_t)n * D, 0.0);
  L.keys.clear();
  std::unordered_map<std::vector<int32_t>, int32_t, KeyHash> table;
  std::vector<double> y(D), b(D + 1);
  std::vector<int64_t> r0(D);
  std::vector<int> rank(D);
  std::vector<int32_t> key(d);
  for (int64_t i = 0; i < n; ++i) {
    elevate(X + i * d, c, y.data());
    const int rc = enclose(y.data(), d, r0.data(), rank.data(), b.data());
    if (rc) return rc;
    for (int k = 0; k <= d; ++k) {
      vertex_key(r0.data(), rank.data(), d, k, key.data());
      auto it = table.find(key);
      int32_t j;
      if (it == table.end()) {
        j = (int32_t)L.m++;
        table.emplace(key, j);
        L.keys.insert(L.keys.end(), key.begin(), key.end());
      } else {
        j = it->second;
      }
      L.idx[i * D + k] = j;
      L.w[i * D + k] = b[k];
    }
  }
  // Neighbours along direction k at t steps: key + t (1 - (d+1) e_k); on the
  // stored coordinates that is +t everywhere except -t*d at coordinate k.
  const int T = 2 * r;
  L.nbr.assign((size_t)L.m * D * T, -1);
  for (int64_t j = 0; j < L.m; ++j) {
    for (int k = 0; k <= d; ++k) {
      int ti = 0;
      for (int t = -r; t <= r; ++t) {
        if (t == 0) continue;
        for (int i = 0; i < d; ++i) {
          const int64_t v = (int64_t)L.keys[j * d + i] + (i == k ? -(int64_t)t * d : (int64_t)t);
          key[i] = (int32_t)v;
        }
        auto it = table.find(key);
        L.nbr[(j * D + k) * T + ti] = (it == table.end()) ? -1 : it->second;
        ++ti;
      }
    }
  }
  return 0;
}

// U (m x C) <- W^T V
void splat(const Lattice& L, const double* V, int C, std::vector<double>& U) {
  const int D = L.c.d + 1;
  U.assign((size_t)L.m * C, 0.0);
  for (int64_t i = 0; i < L.n; ++i)
    for (int k = 0; k < D; ++k) {
      const int32_t j = L.idx[i * D + k];
      const double wk = L.w[i * D + k];
      for (int c = 0; c < C; ++c) U[(size_t)j * C + c] += wk * V[i * C + c];
    }
}

// One direction of the blur: U'[j] = sum_t stencil[t] U[neighbour(j, k, t)].
void blur_direction(const Lattice& L, int k, const std::vector<double>& U, int C,
                    std::vector<double>& out) {
  const int D = L.c.d + 1, r = L.c.r, T = 2 * r;
  out.assign(U.size(), 0.0);
  for (int64_t j = 0; j < L.m; ++j) {
    for (int c = 0; c < C; ++c) {
      double acc = 0.0;
      int ti = 0;
      for (int t = -r; t <= r; ++t) {
        double u;
        if (t == 0) {
          u = U[(size_t)j * C + c];
        } else {
          const int32_t nb = L.nbr[(j * D + k) * T + ti];
          u = nb >= 0 ? U[(size_t)nb * C + c] : 0.0;
          ++ti;
        }
        acc += L.c.stencil[t + r] * u;
      }
      out[(size_t)j * C + c] = acc;
    }
  }
}

void blur(const Lattice& L, std::vector<double>& U, int C, int mode) {
  const int d = L.c.d;
  std::vector<double> tmp;
  if (mode == ORC_BLUR_FORWARD || mode == ORC_BLUR_REVERSE) {
    for (int s = 0; s <= d; ++s) {
      const int k = (mode == ORC_BLUR_FORWARD) ? s : d - s;
      blur_direction(L, k, U, C, tmp);
      U.swap(tmp);
    }
    return;
  }
  std::vector<double> F = U, R = U;
  blur(L, F, C, ORC_BLUR_FORWARD);
  blur(L, R, C, ORC_BLUR_REVERSE);
  for (size_t q = 0; q < U.size(); ++q) U[q] = 0.5 * (F[q] + R[q]);
}

// out (n x C) <- scale * W U
void slice(const Lattice& L, const std::vector<double>& U, int C, double scale, double* out) {
  const int D = L.c.d + 1;
  for (int64_t i = 0; i < L.n; ++i)
    for (int c = 0; c < C; ++c) {
      double acc = 0.0;
      for (int k = 0; k < D; ++k)
        acc += L.w[i * D + k] * U[(size_t)L.idx[i * D + k] * C + c];
      out[i * C + c] = scale * acc;
    }
}

void mvm(const Lattice& L, const double* V, int C, int mode, double os, double* out) {
  std::vector<double> U;
  splat(L, V, C, U);
  blur(L, U, C, mode);
  slice(L, U, C, os, out);
}

bool valid_mode(int mode) {
  return mode == ORC_BLUR_SYMMETRIC || mode == ORC_BLUR_FORWARD || mode == ORC_BLUR_REVERSE;
}

}  // namespace

extern "C" {

int orc_constants(int d, int r, int kernel, const double* ell, double* s, double* stencil,
                  double* alpha, double* f) {
  Consts c;
  const int rc = make_consts(d, r, kernel, ell, c);
  if (rc) return rc;
  if (s) *s = c.s;
  if (alpha) *alpha = c.alpha;
  if (stencil) std::memcpy(stencil, c.stencil.data(), sizeof(double) * c.stencil.size());
  if (f) std::memcpy(f, c.f.data(), sizeof(double) * d);
  return 0;
}

int orc_embed(const float* X, int64_t n, int d, const double* ell, int r, int kernel, double* y) {
  Consts c;
  if (make_consts(d, r, kernel, ell, c) || n < 0 || !X || !y) return -1;
  for (int64_t i = 0; i < n; ++i) elevate(X + i * d, c, y + i * (d + 1));
  return 0;
}

int orc_simplex(const float* X, int64_t n, int d, const double* ell, int r, int kernel,
                int32_t* keys, double* bary, int32_t* r0_out, int32_t* rank_out) {
  Consts c;
  if (make_consts(d, r, kernel, ell, c) || n < 0 || !X) return -1;
  const int D = d + 1;
  std::vector<double> y(D), b(D + 1);
  std::vector<int64_t> r0(D);
  std::vector<int> rank(D);
  for (int64_t i = 0; i < n; ++i) {
    elevate(X + i * d, c, y.data());
    const int rc = enclose(y.data(), d, r0.data(), rank.data(), b.data());
    if (rc) return rc;
    for (int k = 0; k < D; ++k) {
      if (keys) vertex_key(r0.data(), rank.data(), d, k, keys + (i * D + k) * d);
      if (bary) bary[i * D + k] = b[k];
      if (r0_out) r0_out[i * D + k] = (int32_t)r0[k];
      if (rank_out) rank_out[i * D + k] = rank[k];
    }
  }
  return 0;
}

void* orc_build(const float* X, int64_t n, int d, const double* ell, int r, int kernel) {
  Consts c;
  if (make_consts(d, r, kernel, ell, c) || n < 1 || !X) return nullptr;
  Lattice* L = new Lattice();
  if (build_lattice(X, n, c, *L)) { delete L; return nullptr; }
  return L;
}

int64_t orc_num_vertices(const void* lat) {
  return lat ? static_cast<const Lattice*>(lat)->m : -1;
}

int orc_export(const void* lat, int32_t* keys, int32_t* idx, double* w, int32_t* nbr) {
  if (!lat) return -1;
  const Lattice& L = *static_cast<const Lattice*>(lat);
  if (keys) std::memcpy(keys, L.keys.data(), sizeof(int32_t) * L.keys.size());
  if (idx) std::memcpy(idx, L.idx.data(), sizeof(int32_t) * L.idx.size());
  if (w) std::memcpy(w, L.w.data(), sizeof(double) * L.w.size());
  if (nbr) std::memcpy(nbr, L.nbr.data(), sizeof(int32_t) * L.nbr.size());
  return 0;
}

void orc_free(void* lat) { delete static_cast<Lattice*>(lat); }

int orc_mvm(const void* lat, const double* V, int C, int mode, double os, double* out) {
  if (!lat || !V || !out || C < 1 || !valid_mode(mode)) return -1;
  mvm(*static_cast<const Lattice*>(lat), V, C, mode, os, out);
  return 0;
}

int orc_splat(const void* lat, const double* V, int C, double* U) {
  if (!lat || !V || !U || C < 1) return -1;
  const Lattice& L = *static_cast<const Lattice*>(lat);
  std::vector<double> tmp;
  splat(L, V, C, tmp);
  std::memcpy(U, tmp.data(), sizeof(double) * tmp.size());
  return 0;
}

int orc_slice(const void* lat, const double* U, int C, double* out) {
  if (!lat || !U || !out || C < 1) return -1;
  const Lattice& L = *static_cast<const Lattice*>(lat);
  std::vector<double> tmp(U, U + (size_t)L.m * C);
  slice(L, tmp, C, 1.0, out);
  return 0;
}

int orc_blur(const void* lat, double* U, int C, int mode) {
  if (!lat || !U || C < 1 || !valid_mode(mode)) return -1;
  const Lattice& L = *static_cast<const Lattice*>(lat);
  std::vector<double> tmp(U, U + (size_t)L.m * C);
  blur(L, tmp, C, mode);
  std::memcpy(U, tmp.data(), sizeof(double) * tmp.size());
  return 0;
}

// Conjugate gradients (Hestenes-Stiefel form), one independent recurrence per
// column of B; a column stops once its recursive residual norm reaches tol
// relative to ||b|| and is left unchanged afterwards. With rows > 0 only the
// first `rows` points take part: the operator is the lattice operator
// restricted to them (the other points splat zero and are not solved for).
int orc_cg_rows(const void* lat, const double* B, int C, int mode, double os, double noise,
                double tol, int max_iter, int64_t rows, double* X, int32_t* iters,
                double* rel_rec, double* rel_true) {
  if (!lat || !B || !X || C < 1 || !valid_mode(mode) || max_iter < 1 || !(noise >= 0.0) ||
      !(tol >= 0.0))
    return -1;
  const Lattice& L = *static_cast<const Lattice*>(lat);
  const int64_t N = L.n;
  const int64_t n = (rows > 0 && rows < N) ? rows : N;
  std::vector<double> x(n), r(n), p(N, 0.0), q(N);
  auto apply = [&](const std::vector<double>& in, std::vector<double>& out) {
    mvm(L, in.data(), 1, mode, os, out.data());
    for (int64_t i = 0; i < n; ++i) out[i] += noise * in[i];
  };
  for (int c = 0; c < C; ++c) {
    double bb = 0.0;
    for (int64_t i = 0; i < n; ++i) bb += B[i * C + c] * B[i * C + c];
    const double bnorm = std::sqrt(bb);
    for (int64_t i = 0; i < n; ++i) { x[i] = 0.0; r[i] = B[i * C + c]; p[i] = r[i]; }
    double rr = bb;
    int it = 0;
    double rel = bnorm > 0.0 ? 1.0 : 0.0;
    while (bnorm > 0.0 && it < max_iter) {
      apply(p, q);
      double pq = 0.0;
      for (int64_t i = 0; i < n; ++i) pq += p[i] * q[i];
      const double alpha = rr / pq;
      for (int64_t i = 0; i < n; ++i) x[i] += alpha * p[i];
      for (int64_t i = 0; i < n; ++i) r[i] -= alpha * q[i];
      double rr_new = 0.0;
      for (int64_t i = 0; i < n; ++i) rr_new += r[i] * r[i];
      ++it;
      rel = std::sqrt(rr_new) / bnorm;
      if (rel <= tol) break;
      const double beta = rr_new / rr;
      for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
      rr = rr_new;
    }
    for (int64_t i = 0; i < N; ++i) X[i * C + c] = i < n ? x[i] : 0.0;
    if (iters) iters[c] = it;
    if (rel_rec) rel_rec[c] = rel;
    if (rel_true) {
      if (bnorm > 0.0) {
        std::vector<double> xf(N, 0.0);
        for (int64_t i = 0; i < n; ++i) xf[i] = x[i];
        apply(xf, q);
        double res = 0.0;
        for (int64_t i = 0; i < n; ++i) {
          const double e = B[i * C + c] - q[i];
          res += e * e;
        }
        rel_true[c] = std::sqrt(res) / bnorm;
      } else {
        rel_true[c] = 0.0;
      }
    }
  }
  return 0;
}

int orc_cg(const void* lat, const double* B, int C, int mode, double os, double noise,
           double tol, int max_iter, double* X, int32_t* iters, double* rel_rec,
           double* rel_true) {
  return orc_cg_rows(lat, B, C, mode, os, noise, tol, max_iter, 0, X, iters, rel_rec, rel_true);
}

// Gradient of L = sum G .* (K V) with respect to the scaled inputs z = x / l,
// following Section 4.2: with k' the derivative of the kernel with respect to
// the squared distance,
//   dL/dz_n = 2 sum_j k'_nj (z_n - z_j) (g_n v_j + v_n g_j)   (summed over channels)
//           = 2 [ g_n (z_n (K'v)_n - (K'(z v))_n) + v_n (z_n (K'g)_n - (K'(z g))_n) ],
// so one filtering of the channels [v, z*v, g, z*g] with K' gives it. For the
// RBF kernel k' = -k/2, so K' is -1/2 times the lattice operator itself.
int orc_mvm_grad(const float* X, int64_t n, int d, const double* ell, int r, int kernel,
                 int mode, const double* V, const double* G, int C, double* dX,
                 double* dlogell) {
  if (kernel != ORC_KERNEL_RBF || !X || !V || !G || C < 1 || !valid_mode(mode)) return -1;
  Consts c;
  if (make_consts(d, r, kernel, ell, c) || n < 1) return -1;
  Lattice L;
  const int rc = build_lattice(X, n, c, L);
  if (rc) return rc;
  const int D = d + 1;
  const int CH = 2 * C * D;  // per channel c: v, z_1 v .. z_d v, g, z_1 g .. z_d g
  std::vector<double> in((size_t)n * CH), out((size_t)n * CH);
  for (int64_t i = 0; i < n; ++i)
    for (int cc = 0; cc < C; ++cc) {
      double* row = &in[(size_t)i * CH + (size_t)cc * 2 * D];
      const double v = V[i * C + cc], g = G[i * C + cc];
      row[0] = v;
      row[D] = g;
      for (int p = 0; p < d; ++p) {
        const double z = (double)X[i * d + p] / ell[p];
        row[1 + p] = z * v;
        row[D + 1 + p] = z * g;
      }
    }
  mvm(L, in.data(), CH, mode, -0.5, out.data());  // K' = -K/2
  std::vector<double> dz(d);
  if (dlogell) for (int p = 0; p < d; ++p) dlogell[p] = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    for (int p = 0; p < d; ++p) dz[p] = 0.0;
    for (int cc = 0; cc < C; ++cc) {
      const double* o = &out[(size_t)i * CH + (size_t)cc * 2 * D];
      const double v = V[i * C + cc], g = G[i * C + cc];
      for (int p = 0; p < d; ++p) {
        const double z = (double)X[i * d + p] / ell[p];
        dz[p] += 2.0 * (g * (z * o[0] - o[1 + p]) + v * (z * o[D] - o[D + 1 + p]));
      }
    }
    for (int p = 0; p < d; ++p) {
      const double z = (double)X[i * d + p] / ell[p];
      if (dX) dX[i * d + p] = dz[p] / ell[p];
      if (dlogell) dlogell[p] -= z * dz[p];
    }
  }
  return 0;
}

}  // extern "C"
