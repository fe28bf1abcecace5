// The lattice MVM  out = outputscale * W_X K_UU W_X^T V  (Section 4, eq. ski_to_bf):
//   k_splat  U = W^T V: every (point, vertex) adds w * V[point] into its
//            lattice row with a float atomic (Section 3.2, Splat)
//   k_blur   one step of the blur: U'[j] = sum_t stencil[t] U[nbr(j, k, t)],
//            missing neighbours contributing zero (Section 3.2, Blur); in
//            SYMMETRIC order the forward chain (direction step) and the
//            reverse chain (direction d-step) advance in the same launch
//   k_slice  out = scale * W U, gathering the d+1 vertex rows of every point
//            (Section 3.2, Slice); the CG variant also adds noise * p and
//            emits per-block partial sums of p . out per column
//
// Layout: point-side arrays are n x C row-major, lattice values m x C
// row-major, so the G lanes that share one row (G = the power of two >= C,
// at most 64) read and write it contiguously.
#include "sgp_internal.h"

namespace sgp {
namespace {

template <int G>
__global__ __launch_bounds__(kBlock) void k_splat(const int32_t* __restrict__ idx,
                                                  const float* __restrict__ w,
                                                  const float* __restrict__ V,
                                                  float* __restrict__ U, int64_t n, int D, int C) {
  constexpr int R = kBlock / G;
  const int lane = threadIdx.x % G;
  const int64_t stride = (int64_t)gridDim.x * R;
  for (int64_t i = (int64_t)blockIdx.x * R + threadIdx.x / G; i < n; i += stride) {
    const int32_t* ii = idx + i * D;
    const float* wi = w + i * D;
    for (int c = lane; c < C; c += G) {
      const float v = V[i * C + c];
      for (int k = 0; k < D; ++k) unsafeAtomicAdd(&U[(int64_t)ii[k] * C + c], wi[k] * v);
    }
  }
}

struct BlurArgs {
  const float* in[2];
  float* out[2];
  const int32_t* nbr[2];  // neighbour table of this step's direction, per chain
  int64_t m;
  int C;
  int r;
  int chains;
  float st[2 * kMaxOrder + 1];
};

template <int G>
__global__ __launch_bounds__(kBlock) void k_blur(BlurArgs a) {
  constexpr int R = kBlock / G;
  const int lane = threadIdx.x % G;
  const int64_t rows = a.m * a.chains;
  const int64_t stride = (int64_t)gridDim.x * R;
  const int C = a.C, r = a.r;
  for (int64_t q = (int64_t)blockIdx.x * R + threadIdx.x / G; q < rows; q += stride) {
    const int ch = q >= a.m ? 1 : 0;
    const int64_t j = q - (ch ? a.m : 0);
    const float* in = a.in[ch];
    const int32_t* nb = a.nbr[ch] + j;
    for (int c = lane; c < C; c += G) {
      float acc = 0.f;
      int ti = 0;
      for (int t = -r; t <= r; ++t) {
        float u;
        if (t == 0) {
          u = in[j * C + c];
        } else {
          const int32_t x = nb[(int64_t)ti * a.m];
          u = x >= 0 ? in[(int64_t)x * C + c] : 0.f;
          ++ti;
        }
        acc = __builtin_fmaf(a.st[t + r], u, acc);
      }
      a.out[ch][j * C + c] = acc;
    }
  }
}

template <int G, bool SYM, bool CG>
__global__ __launch_bounds__(kBlock) void k_slice(const int32_t* __restrict__ idx,
                                                  const float* __restrict__ w,
                                                  const float* __restrict__ UF,
                                                  const float* __restrict__ UR,
                                                  float* __restrict__ out, int64_t n, int D, int C,
                                                  float scale, float noise,
                                                  const float* __restrict__ p,
                                                  double* __restrict__ partials) {
  constexpr int R = kBlock / G;
  const int lane = threadIdx.x % G;
  const int64_t stride = (int64_t)gridDim.x * R;
  double dot = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * R + threadIdx.x / G; i < n; i += stride) {
    const int32_t* ii = idx + i * D;
    const float* wi = w + i * D;
    for (int c = lane; c < C; c += G) {
      float acc = 0.f;
      for (int k = 0; k < D; ++k) {
        const int64_t row = (int64_t)ii[k] * C + c;
        float u = UF[row];
        if (SYM) u += UR[row];
        acc = __builtin_fmaf(wi[k], u, acc);
      }
      float o = scale * acc;
      if (CG) {
        const float pv = p[i * C + c];
        o = __builtin_fmaf(noise, pv, o);
        dot += (double)pv * (double)o;
      }
      out[i * C + c] = o;
    }
  }
  if (CG) {
    __shared__ double sh[kBlock];
    sh[threadIdx.x] = dot;
    __syncthreads();
    if ((int)threadIdx.x < C) {
      double s = 0.0;
      for (int rr = 0; rr < R; ++rr) s += sh[rr * G + threadIdx.x];
      partials[(int64_t)blockIdx.x * C + threadIdx.x] = s;
    }
  }
}

unsigned grid_rows(int64_t rows, int G, int64_t cap) {
  const int64_t R = kBlock / G;
  int64_t b = (rows + R - 1) / R;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

template <int G>
int launch_splat(const sgp_lattice* L, const float* V, int C, float* U, hipStream_t s) {
  ProfScope ps(KK_SPLAT, s);
  hipLaunchKernelGGL(k_splat<G>, dim3(grid_rows(L->n, G, 32768)), dim3(kBlock), 0, s,
                     (const int32_t*)L->idx.ptr, (const float*)L->w.ptr, V, U, L->n, L->d + 1, C);
  SGP_LAUNCH_CHECK("k_splat");
  return SGP_OK;
}

template <int G>
int launch_blur(const BlurArgs& a, hipStream_t s) {
  ProfScope ps(KK_BLUR, s);
  hipLaunchKernelGGL(k_blur<G>, dim3(grid_rows(a.m * a.chains, G, 32768)), dim3(kBlock), 0, s, a);
  SGP_LAUNCH_CHECK("k_blur");
  return SGP_OK;
}

template <int G, bool SYM, bool CG>
int launch_slice(const sgp_lattice* L, const float* UF, const float* UR, float* out, int C,
                 float scale, float noise, const float* p, double* partials, hipStream_t s) {
  ProfScope ps(KK_SLICE, s);
  const unsigned grid = CG ? (unsigned)kRedBlocks : grid_rows(L->n, G, 32768);
  hipLaunchKernelGGL((k_slice<G, SYM, CG>), dim3(grid), dim3(kBlock), 0, s,
                     (const int32_t*)L->idx.ptr, (const float*)L->w.ptr, UF, UR, out, L->n,
                     L->d + 1, C, scale, noise, p, partials);
  SGP_LAUNCH_CHECK("k_slice");
  return SGP_OK;
}

template <int G>
int mvm_g(const sgp_lattice* L, const float* V, int C, float* out, hipStream_t s, float noise,
          const float* p, double* partials) {
  const int d = L->d, T = 2 * L->order;
  const int64_t m = L->m, mC = m * C;
  float* U0 = (float*)L->ubuf.ptr;
  float* B1 = U0 + mC;
  float* B2 = B1 + mC;
  float* B3 = B2 + mC;
  int rc;
  if ((rc = launch_fill_u32((uint32_t*)U0, (size_t)mC, 0u, s))) return rc;
  if ((rc = launch_splat<G>(L, V, C, U0, s))) return rc;

  const bool sym = L->blur == SGP_BLUR_SYMMETRIC;
  BlurArgs a;
  a.m = m;
  a.C = C;
  a.r = L->order;
  a.chains = sym ? 2 : 1;
  for (int t = 0; t < 2 * L->order + 1; ++t) a.st[t] = L->stencil[t];
  const int32_t* nbr = (const int32_t*)L->nbr.ptr;
  const float* cur[2] = {U0, U0};
  for (int step = 0; step <= d; ++step) {
    // chain 0: forward (or the single requested order); chain 1: reverse
    const int k0 = (L->blur == SGP_BLUR_REVERSE) ? d - step : step;
    const int k1 = d - step;
    float* dst0 = (step % 2 == 0) ? B1 : B2;
    float* dst1 = (step % 2 == 0) ? B3 : U0;
    a.in[0] = cur[0];
    a.out[0] = dst0;
    a.nbr[0] = nbr + (int64_t)k0 * T * m;
    a.in[1] = cur[1];
    a.out[1] = dst1;
    a.nbr[1] = nbr + (int64_t)k1 * T * m;
    if ((rc = launch_blur<G>(a, s))) return rc;
    cur[0] = dst0;
    cur[1] = dst1;
  }
  const bool cg = partials != nullptr;
  const float scale = sym ? 0.5f * L->outputscale : L->outputscale;
  if (sym) {
    return cg ? launch_slice<G, true, true>(L, cur[0], cur[1], out, C, scale, noise, p, partials, s)
              : launch_slice<G, true, false>(L, cur[0], cur[1], out, C, scale, 0.f, nullptr, nullptr, s);
  }
  return cg ? launch_slice<G, false, true>(L, cur[0], nullptr, out, C, scale, noise, p, partials, s)
            : launch_slice<G, false, false>(L, cur[0], nullptr, out, C, scale, 0.f, nullptr, nullptr, s);
}

}  // namespace

int mvm_into(const sgp_lattice* L, const float* V, int C, float* out, hipStream_t s, float noise,
             const float* p, double* partials) {
  int rc = dev_reserve(const_cast<sgp_lattice*>(L)->ubuf, sizeof(float) * 4 * L->m * C);
  if (rc) return rc;
  switch (lanes_for(C)) {
    case 1: return mvm_g<1>(L, V, C, out, s, noise, p, partials);
    case 2: return mvm_g<2>(L, V, C, out, s, noise, p, partials);
    case 4: return mvm_g<4>(L, V, C, out, s, noise, p, partials);
    case 8: return mvm_g<8>(L, V, C, out, s, noise, p, partials);
    case 16: return mvm_g<16>(L, V, C, out, s, noise, p, partials);
    case 32: return mvm_g<32>(L, V, C, out, s, noise, p, partials);
    default: return mvm_g<64>(L, V, C, out, s, noise, p, partials);
  }
}

}  // namespace sgp

using namespace sgp;

extern "C" int lattice_mvm(const sgp_lattice* L, const float* values, int32_t C, float* out,
                           void* stream) {
  if (!L || !values || !out) {
    set_error("lattice_mvm: NULL argument");
    return SGP_EINVAL;
  }
  if (C < 1) {
    set_error("lattice_mvm: C must be >= 1 (got %d)", (int)C);
    return SGP_EINVAL;
  }
  const size_t bytes = sizeof(float) * (size_t)L->n * (size_t)C;
  const char* v0 = (const char*)values;
  const char* o0 = (const char*)out;
  if (v0 < o0 + bytes && o0 < v0 + bytes) {
    set_error("lattice_mvm: out overlaps values");
    return SGP_EINVAL;
  }
  return mvm_into(L, values, C, out, (hipStream_t)stream, 0.f, nullptr, nullptr);
}
