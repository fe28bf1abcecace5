// Gradient of L = sum_{i,c} G[i,c] (outputscale * K V)[i,c] with respect to
// the points and the log-lengthscales, by filtering (Section 4.2).
//
// With z = x / l and k' the derivative of the kernel with respect to the
// squared distance,
//   dL/dz_n = 2 sum_j k'_nj (z_n - z_j) (g_n v_j + v_n g_j)
//           = 2 [ g_n (z_n (K'v)_n - (K'(z v))_n) + v_n (z_n (K'g)_n - (K'(z g))_n) ],
// so one filtering of the 2(d+1) channels [v, z*v, g, z*g] per input column
// gives it. For the RBF kernel k' = -k/2, so K' is -1/2 times the lattice
// operator. Then dL/dx = dL/dz / l and dL/dlog l_p = -sum_n z_np dL/dz_np.
//
// Everything runs in the lattice's internal point order. The channels are
// formed and combined in fp64 and filtered in fp32 (as the forward MVM:
// fp32 weights and values, fp32 lattice accumulation). The columns are taken
// kb at a time (kb * 2(d+1) <= 128 channels), whose channels are filtered
// in blocks of W: all of them in one MVM on a small lattice, narrower blocks
// on a large one, so that the blur's two lattice arrays (m x W) stay within
// the Infinity Cache. An MVM's value for a channel does not depend on the
// other channels, so the results do not depend on W.
#include <algorithm>
#include <cmath>
#include <vector>

#include "sgp_internal.h"

namespace sgp {
namespace {

struct InvEll {
  double v[kMaxD];
};

// Channel bj of point i in blocks of W channels: [bj / W][i][bj % W].
__host__ __device__ inline int64_t chan_at(int64_t n, int W, int64_t i, int bj) {
  return (int64_t)(bj / W) * n * W + i * W + bj % W;
}

// Channel bj = b * 2(d+1) + j, j < 2(d+1), of column c0 + b (b < kb): v,
// z_1 v .. z_d v, g, z_1 g .. z_d g, formed in fp64 and stored in fp32 at
// chan_at; channels past kb * 2(d+1) up to nblk * W are zero.
__global__ __launch_bounds__(kBlock) void k_grad_channels(const float* __restrict__ X,
                                                          const float* __restrict__ V,
                                                          const float* __restrict__ G,
                                                          const uint32_t* __restrict__ perm,
                                                          int64_t n, int d, int C, int c0, int kb,
                                                          int W, int nblk, InvEll ie,
                                                          float* __restrict__ H) {
  const int D = d + 1, CH = 2 * D, K = kb * CH, KW = nblk * W;
  const int64_t total = n * KW;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += stride) {
    const int64_t i = q / KW;
    const int bj = (int)(q - i * KW);
    float h = 0.f;
    if (bj < K) {
      const int b = bj / CH, j = bj - b * CH;
      const int64_t src = perm[i];
      const int half = j < D ? 0 : 1;
      const int jj = j - half * D;
      const int c = c0 + b;
      const double a = half ? (double)G[src * C + c] : (double)V[src * C + c];
      h = (float)(jj == 0 ? a : a * ((double)X[src * d + (jj - 1)] * ie.v[jj - 1]));
    }
    H[chan_at(n, W, i, bj)] = h;
  }
}

// dz[i][p] += -(g (z Kv - Kzv) + v (z Kg - Kzg)) with K = outputscale * K_lat
// (the factor 2 of the derivative and the -1/2 of k' cancel), for columns
// c0 .. c0 + kb - 1 in order, in fp64.
__global__ __launch_bounds__(kBlock) void k_grad_accum(const float* __restrict__ X,
                                                       const float* __restrict__ V,
                                                       const float* __restrict__ G,
                                                       const uint32_t* __restrict__ perm,
                                                       const float* __restrict__ O, int64_t n,
                                                       int d, int C, int c0, int kb, int W, InvEll ie,
                                                       double* __restrict__ dz) {
  const int D = d + 1, CH = 2 * D;
  const int64_t total = n * d;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += stride) {
    const int64_t i = q / d;
    const int p = (int)(q - i * d);
    const int64_t src = perm[i];
    const double z = (double)X[src * d + p] * ie.v[p];
    double acc = dz[q];
    for (int b = 0; b < kb; ++b) {
      const double v = V[src * C + c0 + b], g = G[src * C + c0 + b];
      const int bj = b * CH;
      const double o0 = O[chan_at(n, W, i, bj)], op = O[chan_at(n, W, i, bj + 1 + p)];
      const double oD = O[chan_at(n, W, i, bj + D)], oDp = O[chan_at(n, W, i, bj + D + 1 + p)];
      acc -= g * (z * o0 - op) + v * (z * oD - oDp);
    }
    dz[q] = acc;
  }
}

// dX in the caller's order; t = -z * dz in place of dz (summed per column
// afterwards for the log-lengthscales).
__global__ __launch_bounds__(kBlock) void k_grad_final(const float* __restrict__ X,
                                                       const uint32_t* __restrict__ perm, int64_t n,
                                                       int d, InvEll ie, double* __restrict__ dz,
                                                       float* __restrict__ dX) {
  const int64_t total = n * d;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += stride) {
    const int64_t i = q / d;
    const int p = (int)(q - i * d);
    const int64_t src = perm[i];
    const double z = (double)X[src * d + p] * ie.v[p];
    const double g = dz[q];
    if (dX) dX[src * d + p] = (float)(g * ie.v[p]);
    dz[q] = -z * g;
  }
}

// Column sums of an nrows x ncols fp64 array (ncols <= 32): block b sums a
// contiguous row range; thread (g, col) takes rows g, g + RG, ... of it and
// the RG group sums are folded in order.
constexpr int kColBlocks = 512;
__global__ __launch_bounds__(kBlock) void k_colsum(const double* __restrict__ a, int64_t nrows,
                                                   int ncols, int64_t rows_per_block,
                                                   double* __restrict__ part) {
  __shared__ double sh[kBlock];
  const int RG = kBlock / ncols;
  const int g = threadIdx.x / ncols, col = threadIdx.x - g * ncols;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < nrows ? r0 + rows_per_block : nrows;
  double s = 0.0;
  if (g < RG)
    for (int64_t r = r0 + g; r < r1; r += RG) s += a[r * ncols + col];
  sh[threadIdx.x] = s;
  __syncthreads();
  if ((int)threadIdx.x < ncols) {
    double v = 0.0;
    for (int gg = 0; gg < RG; ++gg) v += sh[gg * ncols + threadIdx.x];
    part[(int64_t)blockIdx.x * ncols + threadIdx.x] = v;
  }
}

unsigned grid_for_g(int64_t work) {
  int64_t b = (work + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > 16384) b = 16384;
  return (unsigned)b;
}

}  // namespace
}  // namespace sgp

using namespace sgp;

extern "C" int lattice_mvm_grad(const sgp_lattice* L, const float* X, const float* V, const float* G,
                                int32_t C, float* dX, double* dlogell, void* stream) {
  if (!L || !X || !V || !G) {
    set_error("lattice_mvm_grad: NULL argument");
    return SGP_EINVAL;
  }
  if (C < 1) {
    set_error("lattice_mvm_grad: C must be >= 1");
    return SGP_EINVAL;
  }
  if (L->kernel != SGP_KERNEL_RBF) {
    set_error("lattice_mvm_grad: only the RBF kernel (k' = -k/2) is supported");
    return SGP_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  const int d = L->d, D = d + 1, CH = 2 * D;
  const int64_t n = L->n;
  InvEll ie;
  for (int p = 0; p < kMaxD; ++p) ie.v[p] = p < d ? 1.0 / L->ell[p] : 0.0;

  void* bufs[4] = {};
  struct Guard {
    void** b;
    hipStream_t s;
    ~Guard() {
      for (int k = 0; k < 4; ++k)
        if (b[k]) dev_release(b[k], s);
    }
  } guard{bufs, s};
  const int kb = std::max(1, std::min((int)C, 128 / CH));  // columns per batch
  // channels per MVM: all of a batch's, unless the blur's two lattice arrays
  // of m x W fp32 would outgrow 320 MiB, a little past the 256 MiB Infinity
  // Cache (a blur launch costs about the same for 8 as for 16 channels, so
  // the widest block whose arrays stay near the cache's size is fastest)
  int W = 64;
  while (W > 4 && 2.0 * (double)L->m * W * sizeof(float) > 320.0 * (1 << 20)) W >>= 1;
  if (W >= kb * CH) W = kb * CH;
  const int nblk_max = (kb * CH + W - 1) / W;
  const size_t hbytes = sizeof(float) * (size_t)n * nblk_max * W;
  const size_t sizes[4] = {hbytes, hbytes, sizeof(double) * n * d, sizeof(double) * kColBlocks * d};
  for (int k = 0; k < 4; ++k) {
    hipError_t e = pool_alloc(&bufs[k], sizes[k], s);
    if (e != hipSuccess) {
      bufs[k] = nullptr;
      (void)hipGetLastError();
      set_error("lattice_mvm_grad: device allocation of %zu bytes failed", sizes[k]);
      return e == hipErrorOutOfMemory ? SGP_ENOMEM : SGP_EHIP;
    }
  }
  float* H = (float*)bufs[0];
  float* O = (float*)bufs[1];
  double* dz = (double*)bufs[2];
  double* part = (double*)bufs[3];
  const uint32_t* perm = (const uint32_t*)L->perm.ptr;
  int rc;
  if ((rc = launch_fill_u32((uint32_t*)dz, (size_t)n * d * 2, 0u, s))) return rc;
  for (int c0 = 0; c0 < C; c0 += kb) {
    const int nb = std::min(kb, (int)C - c0);
    const int Wb = W == kb * CH ? nb * CH : W;  // one MVM of exactly the batch's channels
    const int nblk = (nb * CH + Wb - 1) / Wb;
    {
      ProfScope ps(KK_GRAD, s);
      hipLaunchKernelGGL(k_grad_channels, dim3(grid_for_g(n * nblk * Wb)), dim3(kBlock), 0, s, X, V, G,
                         perm, n, d, (int)C, c0, nb, Wb, nblk, ie, H);
      SGP_LAUNCH_CHECK("k_grad_channels");
    }
    for (int k = 0; k < nblk; ++k)
      if ((rc = mvm_f32(L, H + (int64_t)k * n * Wb, Wb, O + (int64_t)k * n * Wb, s))) return rc;
    {
      ProfScope ps(KK_GRAD, s);
      hipLaunchKernelGGL(k_grad_accum, dim3(grid_for_g(n * d)), dim3(kBlock), 0, s, X, V, G, perm, O,
                         n, d, (int)C, c0, nb, Wb, ie, dz);
      SGP_LAUNCH_CHECK("k_grad_accum");
    }
  }
  {
    ProfScope ps(KK_GRAD, s);
    hipLaunchKernelGGL(k_grad_final, dim3(grid_for_g(n * d)), dim3(kBlock), 0, s, X, perm, n, d, ie, dz,
                       dX);
    SGP_LAUNCH_CHECK("k_grad_final");
    const int64_t rpb = (n + kColBlocks - 1) / kColBlocks;
    hipLaunchKernelGGL(k_colsum, dim3(kColBlocks), dim3(kBlock), 0, s, dz, n, d, rpb, part);
    SGP_LAUNCH_CHECK("k_colsum");
  }
  std::vector<double> host((size_t)kColBlocks * d);
  SGP_HIP(hipMemcpyAsync(host.data(), part, sizeof(double) * host.size(), hipMemcpyDeviceToHost, s));
  SGP_HIP(hipStreamSynchronize(s));
  mark_use(L, s);
  if (dlogell) {
    for (int p = 0; p < d; ++p) {
      double acc = 0.0;
      for (int b = 0; b < kColBlocks; ++b) acc += host[(size_t)b * d + p];
      dlogell[p] = acc;
    }
  }
  return SGP_OK;
}
