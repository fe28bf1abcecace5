// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstddef>
#include <vector>

#include "simplexgp.h"

namespace sgp {

constexpr int kBlock = 256;     // threads per block for every kernel
constexpr int kMaxD = 32;       // largest input dimension
constexpr int kMaxOrder = 8;    // largest stencil half-width r
constexpr int kMaxCgCols = 64;  // columns per cg_solve call
constexpr int kRedBlocks = 512; // blocks (and partial sums) of the reducing vector kernels

void set_error(const char* fmt, ...);
int hip_fail(hipError_t e, const char* what, const char* file, int line);

#define SGP_HIP(call)                                                        \
  do {                                                                       \
    hipError_t _e = (call);                                                  \
    if (_e != hipSuccess) return ::sgp::hip_fail(_e, #call, __FILE__, __LINE__); \
  } while (0)

#define SGP_LAUNCH_CHECK(what)                                               \
  do {                                                                       \
    hipError_t _e = hipGetLastError();                                       \
    if (_e != hipSuccess) return ::sgp::hip_fail(_e, what, __FILE__, __LINE__); \
  } while (0)

// Kernel kinds reported by the event profiler.
enum KernelKind {
  KK_FILL = 0,
  KK_SIMPLEX,
  KK_COUNT,
  KK_SCAN,
  KK_COMPACT,
  KK_RESOLVE,
  KK_NEIGHBORS,
  KK_SPLAT,
  KK_BLUR,
  KK_SLICE,
  KK_CG_INIT,
  KK_CG_SCALAR,
  KK_CG_UPDATE,
  KK_CG_DIR,
  KK_CG_OUT,
  KK_NUM
};

// Brackets one launch with events when profiling is on (no-op otherwise).
class ProfScope {
 public:
  ProfScope(int kind, hipStream_t s);
  ~ProfScope();

 private:
  hipEvent_t stop_;
  hipStream_t stream_;
};

// Device buffer with byte accounting.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

int dev_alloc(DevBuf& b, size_t bytes);
void dev_free(DevBuf& b);
// Grow (never shrink) a work buffer; contents are not preserved.
int dev_reserve(DevBuf& b, size_t bytes);

// Lanes that share one row of C channels: the smallest power of two >= C,
// capped at one wavefront.
inline int lanes_for(int C) {
  int g = 1;
  while (g < C && g < 64) g <<= 1;
  return g;
}

}  // namespace sgp

struct sgp_lattice {
  int64_t n = 0;
  int d = 0;
  int order = 1;
  int kernel = SGP_KERNEL_RBF;
  int blur = SGP_BLUR_SYMMETRIC;
  float outputscale = 1.f;
  int64_t m = 0;
  int device = 0;
  double spacing = 0;
  double stencil64[2 * sgp::kMaxOrder + 1] = {};

  sgp::DevBuf idx;   // n x (d+1) int32
  sgp::DevBuf w;     // n x (d+1) fp32
  sgp::DevBuf keys;  // m x d int32
  sgp::DevBuf nbr;   // (d+1) x 2r x m int32: [direction][offset][point]

  // work buffers, grown on demand
  sgp::DevBuf ubuf;   // lattice values, 4 x m x C fp32
  sgp::DevBuf cgvec;  // CG vectors r, p, q: 3 x n x C fp32
  sgp::DevBuf cgred;  // CG partial sums and per-column scalars
};

namespace sgp {
// Host-side constants (Section 4.1 and Section 3.2 Splat).
int make_constants(int d, int r, int kernel, const double* ell, double* spacing,
                   double* stencil, double* f);

// Launchers used across files.
int launch_fill_u32(uint32_t* p, size_t count, uint32_t value, hipStream_t s);
// fp32 values, fp32 lattice accumulation (lattice_mvm)
int mvm_into(const sgp_lattice* L, const float* V, int C, float* out, hipStream_t s);
// fp64 values and accumulation with the CG epilogue: q = A p, partial sums of p.q
int mvm_cg(const sgp_lattice* L, const double* p, int C, double* q, hipStream_t s, double noise,
           double* partials);
}  // namespace sgp
