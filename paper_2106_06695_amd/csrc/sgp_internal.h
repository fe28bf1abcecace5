// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstddef>
#include <vector>

#include "simplexgp.h"

namespace sgp {

constexpr int kBlock = 256;     // threads per block, except the tile kernels
constexpr int kMaxD = 32;       // largest input dimension
constexpr int kMaxOrder = 8;    // largest stencil half-width r
constexpr int kMaxCgCols = 64;  // columns per cg_solve call
constexpr int kRedBlocks = 512; // blocks (and partial sums) of the reducing vector kernels
constexpr int kPiece = 32;      // longest run piece the splat reduces in one go

// Launch-shape knobs of the MVM kernels. Defaults are the measured best on
// MI355X; SGP_LDS_BUDGET, SGP_SLICE_LDS_BUDGET, SGP_TILE_BLOCKS_PER_CU and
// SGP_BLUR_SEQ_MIB in the environment override them (read once per process).
struct Tuning {
  int lds_budget;        // bytes of LDS the splat may stage (one block per CU)
  int slice_lds_budget;  // bytes of LDS the slice may stage (one block per CU)
  int blocks_per_cu;     // resident blocks per CU of the persistent tile kernels (0 = occupancy)
  int blur_seq_mib;      // initial threshold of sgp_blur_seq_bytes in MiB (0: never)
};
const Tuning& tuning();

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
  KK_SPLAT_GATHER,
  KK_BLUR,
  KK_SLICE,
  KK_CG_INIT,
  KK_CG_SCALAR,
  KK_CG_DIR,
  KK_CG_ALPHA,
  KK_CG_OUT,
  KK_GRAD,
  KK_SORT,
  KK_ORDER,
  KK_NUM
};

// True while the event profiler is enabled.
bool profiling();
// Process-wide switch for graph replay of CG iterations.
bool cg_graphs_enabled();
bool blur_fuse_enabled();
// True when the symmetric blur should run its chains one after the other
// for lattice value arrays of `bytes` in all (four arrays).
bool blur_seq_for(double bytes);
bool cg_fuse_enabled();
// A per-thread, per-device stream used only to record graphs.
hipStream_t capture_stream();

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
  size_t bytes = 0;  // requested
  size_t cap = 0;    // allocated (a reused block may be larger)
};

// Device memory is stream-ordered: allocated on the stream of the call that
// first needs it, released on a library-owned stream once the lattice's last
// use (an event recorded at the end of every call) has completed. Nothing in
// the library synchronises the whole device, so lattices driven from
// different streams overlap.
int dev_alloc(DevBuf& b, size_t bytes, hipStream_t s);
// Release a buffer the device is done with (the caller has waited for its
// last use): it is kept for reuse by later allocations of a similar size.
void dev_free(DevBuf& b);
// The same for a raw block of cap bytes from pool_alloc.
void block_give(void* p, size_t cap);
void* block_take(size_t bytes, size_t* cap);
hipStream_t lib_stream();
// Stream-ordered allocation on the current device: from the caller's
// allocator when one is set (sgp_set_allocator), else from the library's
// pool. dev_release returns such a block to the allocator it came from, in
// stream order on s (or at once if the device is done with it).
hipError_t pool_alloc(void** p, size_t bytes, hipStream_t s);
void dev_release(void* p, hipStream_t s);
// Pinned host scratch of at least `bytes` (<= 64 KiB), one per host thread.
void* pinned_scratch(size_t bytes);

// Lanes that share one row of C channels: the smallest power of two >= C,
// capped at one wavefront.
inline int lanes_for(int C) {
  int g = 1;
  while (g < C && g < 64) g <<= 1;
  return g;
}

}  // namespace sgp

// One (vertex, weight) or (point, weight) entry of the interpolation matrix W.
struct sgp_entry {
  int32_t j;
  float w;
};

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
  double ell[sgp::kMaxD] = {};  // lengthscales the lattice was built with
  int64_t solve_rows = 0;       // CG solves on the first solve_rows points only (0 = all)

  // Internal order: points sorted by their remainder-0 lattice point
  // (lexicographic), then by the ranks of their first coordinates (which
  // groups points of one simplex), lattice points numbered by first touch in
  // that order.
  // Sorted points are cut into tiles of tile_points consecutive points (the
  // entries of tile t are entries t*P*(d+1) onwards, in both orders); each
  // tile lists the distinct lattice points it touches ("runs"), which the
  // splat reduces from LDS-staged values and the slice stages into LDS.
  int tile_points = 256;
  int64_t ntiles = 0;
  int64_t nrun = 0;         // total runs over all tiles
  int max_tile_runs = 0;    // longest tile vertex list
  int64_t npiece = 0;       // runs cut into pieces of at most kPiece entries (splat)
  int max_tile_pieces = 0;  // longest tile piece list
  sgp::DevBuf perm;       // n uint32: sorted position -> caller's point index
  sgp::DevBuf loc;        // n(d+1) uint16: run of (sorted point, vertex) within its tile
  sgp::DevBuf ws;         // n(d+1) fp32: barycentric weight, sorted point order
  sgp::DevBuf tile_off;   // ntiles+1 int32: first run of each tile
  sgp::DevBuf tile_verts; // nrun int32: internal lattice point of each run (ascending per tile)
  sgp::DevBuf stile_off;  // ntiles+1 int32: first piece of each tile
  sgp::DevBuf run_rel;    // npiece uint16: first entry of each piece, relative to its tile's entries
  sgp::DevBuf ent_lp;     // n(d+1) uint8: point within its tile, entries grouped by run
  sgp::DevBuf ent_w;      // n(d+1) fp32: weight of each entry, grouped by run
  sgp::DevBuf occ_ptr;    // m+1 int32: first partial row of each lattice point
  sgp::DevBuf row_vert;   // npiece int32: lattice point of each partial row
  sgp::DevBuf run_dst;    // npiece int32: partial row of each piece; a lattice point's
                          //   pieces occupy rows occ_ptr[j] .. occ_ptr[j+1]-1 in piece order
  sgp::DevBuf nbr;        // (d+1) x m x 2r int32: [direction][internal vertex][offset]
  sgp::DevBuf int2can;    // m int32: internal vertex -> canonical index
  sgp::DevBuf keys;       // m x d int32 in canonical order (first occurrence in caller's order)

  hipEvent_t last_use = nullptr;  // recorded at the end of every call on the lattice

  // work buffers, grown on demand
  sgp::DevBuf ubuf;   // lattice values 4 x m x C (5 inside CG), piece partial sums npiece x C, gather fragments
  sgp::DevBuf cgvec;  // CG vectors: r and p (n x C fp64 each), then x (n x C fp32)
  sgp::DevBuf cgred;  // CG partial sums and per-column scalars
};

namespace sgp {
// Grow (never shrink) a work buffer of L; contents are not preserved. Waits
// for L's last use before releasing a smaller buffer.
int dev_reserve(const sgp_lattice* L, DevBuf& b, size_t bytes, hipStream_t s);
// Record the end of a call on L (its last use) on stream s.
void mark_use(const sgp_lattice* L, hipStream_t s);
// Wait for L's last recorded use.
int wait_last_use(const sgp_lattice* L);

// Host-side constants (Section 4.1 and Section 3.2 Splat).
int make_constants(int d, int r, int kernel, const double* ell, double* spacing,
                   double* stencil, double* f);

// Launchers used across files.
int launch_fill_u32(uint32_t* p, size_t count, uint32_t value, hipStream_t s);

// Device-wide exclusive scan (tmp: scan_tmp_words(count) words) and stable
// LSD radix sort of (key, value) pairs on the low `bits` key bits (tmp:
// radix_tmp_words(count) words). The sorted pairs end in the *_alt arrays
// when *result_in_alt is set.
int scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t count, uint32_t* total,
                       uint32_t* tmp, hipStream_t s);
size_t scan_tmp_words(int64_t count);
size_t radix_tmp_words(int64_t count);
template <typename K>
int radix_sort_pairs(K* keys, uint32_t* vals, K* keys_alt, uint32_t* vals_alt, int64_t count,
                     int bits, uint32_t* tmp, hipStream_t s, bool* result_in_alt);
// Forget the build shapes sgp_autotune_build chose.
void build_tune_reset();
// fp32 values, fp32 lattice accumulation (lattice_mvm)
int mvm_into(const sgp_lattice* L, const float* V, int C, float* out, hipStream_t s);
// fp64 values and accumulation inside CG: A p, then alpha, r -= alpha A p
// and beta (CgMvm); up (may be null) is the previous iteration's direction
// update, which the splat applies to p (in place) and x before splatting p
struct CgMvm;
struct CgDirUpdate;
// The CG direction update as a pass of its own over the n x C arrays
int launch_cg_dir(const CgDirUpdate& up, int64_t nC, int C, hipStream_t s);
// alpha of a CG step from the splatted u, the blurred B u (m x C each) and
// the splat's p.p tile rows
int launch_cg_alpha(const double* u, const double* bu, int64_t m, int C, double scale, const CgMvm& cg,
                    hipStream_t s);
int mvm_cg(const sgp_lattice* L, double* p, int C, hipStream_t s, double noise, const CgMvm& cg,
           const CgDirUpdate* up);
// fp64 values and accumulation, internal point order, no epilogue
int mvm_f64(const sgp_lattice* L, const double* V, int C, double* out, hipStream_t s);
// fp32 values and accumulation, internal point order
int mvm_f32(const sgp_lattice* L, const float* V, int C, float* out, hipStream_t s);
}  // namespace sgp
