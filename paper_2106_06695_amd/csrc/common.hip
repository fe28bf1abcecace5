// Errors, allocation, event profiling, host constants and small API calls.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <map>
#include <mutex>
#include <vector>

#include "sgp_internal.h"

namespace sgp {

namespace {
thread_local char g_err[512] = "";

int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  if (!v || !*v) return dflt;
  char* end = nullptr;
  const long x = std::strtol(v, &end, 10);
  return (end && *end == 0) ? (int)x : dflt;
}
}  // namespace

const Tuning& tuning() {
  static const Tuning t = [] {
    Tuning k;
    k.lds_budget = env_int("SGP_LDS_BUDGET", 131072);
    if (k.lds_budget < 16384) k.lds_budget = 16384;
    if (k.lds_budget > 163840) k.lds_budget = 163840;
    k.slice_lds_budget = env_int("SGP_SLICE_LDS_BUDGET", 131072);
    if (k.slice_lds_budget < 16384) k.slice_lds_budget = 16384;
    if (k.slice_lds_budget > 163840) k.slice_lds_budget = 163840;
    k.blocks_per_cu = env_int("SGP_TILE_BLOCKS_PER_CU", 0);
    if (k.blocks_per_cu < 0) k.blocks_per_cu = 0;
    k.blur_seq_mib = env_int("SGP_BLUR_SEQ_MIB", 128);
    if (k.blur_seq_mib < 0) k.blur_seq_mib = 0;
    return k;
  }();
  return t;
}

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int hip_fail(hipError_t e, const char* what, const char* file, int line) {
  set_error("HIP error %d (%s) in %s at %s:%d", (int)e, hipGetErrorString(e), what, file, line);
  return e == hipErrorOutOfMemory ? SGP_ENOMEM : SGP_EHIP;
}

// Device memory comes from the library's stream-ordered pool, or from a
// caller's allocator (sgp_set_allocator). Every block is returned to the
// allocator it came from: the allocator changes only while the library
// holds no block (g_live counts blocks held by lattices, temporaries and
// the gradient, not idle cached ones). The hooks run under g_alloc_mu.
namespace {
std::mutex g_alloc_mu;
void* (*g_user_alloc)(size_t, void*) = nullptr;
void (*g_user_free)(void*, void*) = nullptr;
int64_t g_live = 0;
}  // namespace

bool user_allocator() {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  return g_user_alloc != nullptr;
}

void dev_release(void* p, hipStream_t s) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  --g_live;
  if (g_user_free)
    g_user_free(p, (void*)s);
  else
    (void)hipFreeAsync(p, s);
}

// Idle device blocks kept for reuse, per device, up to a quarter of the
// device memory. Freeing pool memory costs the host about 0.2 ms per block
// on this runtime, so a lattice's ~20 arrays are recycled instead.
namespace {
struct BlockCache {
  std::mutex mu;
  std::multimap<size_t, void*> blocks;
  size_t bytes = 0, limit = 0;
};
BlockCache* block_cache() {
  constexpr int kMaxDevices = 64;
  static BlockCache caches[kMaxDevices];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  return &caches[dev];
}
}  // namespace

void* block_take(size_t bytes, size_t* cap) {
  std::lock_guard<std::mutex> la(g_alloc_mu);
  if (g_user_alloc) return nullptr;  // the caller's allocator does its own caching
  BlockCache* c = block_cache();
  if (!c) return nullptr;
  std::lock_guard<std::mutex> lk(c->mu);
  auto it = c->blocks.lower_bound(bytes);
  if (it == c->blocks.end() || it->first > bytes + bytes / 4 + ((size_t)1 << 20)) return nullptr;
  void* p = it->second;
  *cap = it->first;
  c->bytes -= it->first;
  c->blocks.erase(it);
  ++g_live;
  return p;
}

void block_give(void* p, size_t cap) {
  if (!p) return;
  {
    std::lock_guard<std::mutex> la(g_alloc_mu);
    BlockCache* c = g_user_alloc ? nullptr : block_cache();
    if (c) {
      std::lock_guard<std::mutex> lk(c->mu);
      if (!c->limit) {
        size_t fr = 0, total = 0;
        c->limit = hipMemGetInfo(&fr, &total) == hipSuccess ? total / 4 : ((size_t)1 << 32);
      }
      if (c->bytes + cap <= c->limit) {
        c->blocks.emplace(cap, p);
        c->bytes += cap;
        --g_live;
        return;
      }
    }
  }
  dev_release(p, lib_stream());
}

// Release every idle cached block of every device (before the allocator
// changes). g_alloc_mu is held by the caller.
namespace {
void flush_block_caches() {
  int ndev = 0, cur = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hipGetDevice(&cur) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  for (int dev = 0; dev < ndev && dev < 64; ++dev) {
    if (hipSetDevice(dev) != hipSuccess) continue;
    BlockCache* c = block_cache();
    if (!c) continue;
    std::lock_guard<std::mutex> lk(c->mu);
    for (auto& kv : c->blocks) (void)hipFreeAsync(kv.second, lib_stream());
    c->blocks.clear();
    c->bytes = 0;
  }
  (void)hipSetDevice(cur);
}
}  // namespace

// Release this device's idle cached blocks to the pool and wait until the
// pool can hand their memory out again (on any stream). Returns the bytes
// released.
namespace {
size_t flush_idle_blocks() {
  BlockCache* c = block_cache();
  if (!c) return 0;
  size_t freed = 0;
  {
    std::lock_guard<std::mutex> la(g_alloc_mu);
    std::lock_guard<std::mutex> lk(c->mu);
    for (auto& kv : c->blocks) (void)hipFreeAsync(kv.second, lib_stream());
    freed = c->bytes;
    c->blocks.clear();
    c->bytes = 0;
  }
  if (freed) (void)hipStreamSynchronize(lib_stream());
  (void)hipGetLastError();
  return freed;
}
std::atomic<int> g_inject_oom{0};
}  // namespace

void inject_oom(int count) { g_inject_oom.store(count > 0 ? count : 0); }

void idle_cache_info(int64_t* bytes, int32_t* blocks) {
  BlockCache* c = block_cache();
  int64_t b = 0;
  int32_t k = 0;
  if (c) {
    std::lock_guard<std::mutex> lk(c->mu);
    b = (int64_t)c->bytes;
    k = (int32_t)c->blocks.size();
  }
  if (bytes) *bytes = b;
  if (blocks) *blocks = k;
}

int dev_alloc(DevBuf& b, size_t bytes, hipStream_t s) {
  b.ptr = nullptr;
  b.bytes = 0;
  b.cap = 0;
  if (bytes == 0) return SGP_OK;
  size_t cap = 0;
  if ((b.ptr = block_take(bytes, &cap))) {
    b.bytes = bytes;
    b.cap = cap;
    return SGP_OK;
  }
  hipError_t e = pool_alloc(&b.ptr, bytes, s);
  if (e != hipSuccess) {
    b.ptr = nullptr;
    (void)hipGetLastError();
    set_error("device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? SGP_ENOMEM : SGP_EHIP;
  }
  b.bytes = bytes;
  b.cap = bytes;
  return SGP_OK;
}

// Device memory comes from a library-owned stream-ordered pool per device
// that keeps freed memory for reuse (release threshold: never), so repeated
// builds and frees do not map and unmap device memory each time.
hipMemPool_t lib_pool() {
  constexpr int kMaxDevices = 64;
  static hipMemPool_t pools[kMaxDevices] = {};
  static std::mutex mu;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  if (!pools[dev]) {
    hipMemPoolProps props = {};
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t pool = nullptr;
    if (hipMemPoolCreate(&pool, &props) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    uint64_t keep = ~0ull;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    pools[dev] = pool;
  }
  return pools[dev];
}

namespace {
hipError_t pool_alloc_once(void** p, size_t bytes, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  if (!g_user_alloc) {
    // test hook: report out-of-memory without asking the pool
    int left = g_inject_oom.load();
    while (left > 0 && !g_inject_oom.compare_exchange_weak(left, left - 1)) {
    }
    if (left > 0) return hipErrorOutOfMemory;
  }
  if (g_user_alloc) {
    *p = g_user_alloc(bytes, (void*)s);
    if (!*p) return hipErrorOutOfMemory;
    ++g_live;
    return hipSuccess;
  }
  hipMemPool_t pool = lib_pool();
  const hipError_t e = pool ? hipMallocFromPoolAsync(p, bytes, pool, s) : hipMallocAsync(p, bytes, s);
  if (e == hipSuccess) ++g_live;
  return e;
}
}  // namespace

hipError_t pool_alloc(void** p, size_t bytes, hipStream_t s) {
  hipError_t e = pool_alloc_once(p, bytes, s);
  // Out of memory while idle blocks of other sizes sit in the cache: give
  // them back to the pool and try once more.
  if (e == hipErrorOutOfMemory && !user_allocator()) {
    (void)hipGetLastError();
    if (flush_idle_blocks() > 0) e = pool_alloc_once(p, bytes, s);
  }
  return e;
}

hipStream_t lib_stream() {
  constexpr int kMaxDevices = 64;
  static hipStream_t streams[kMaxDevices] = {};
  static std::mutex mu;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  if (!streams[dev]) {
    // default priority, never blocks on the legacy stream
    if (hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess) streams[dev] = nullptr;
  }
  return streams[dev];
}

void dev_free(DevBuf& b) {
  if (b.ptr) block_give(b.ptr, b.cap);
  b.ptr = nullptr;
  b.bytes = 0;
  b.cap = 0;
}

void* pinned_scratch(size_t bytes) {
  constexpr size_t kBytes = 65536;
  thread_local void* buf = nullptr;
  if (bytes > kBytes) return nullptr;
  if (!buf && hipHostMalloc(&buf, kBytes, hipHostMallocDefault) != hipSuccess) buf = nullptr;
  return buf;
}

int wait_last_use(const sgp_lattice* L) {
  if (L && L->last_use) SGP_HIP(hipEventSynchronize(L->last_use));
  return SGP_OK;
}

void mark_use(const sgp_lattice* L, hipStream_t s) {
  if (L && L->last_use) (void)hipEventRecord(L->last_use, s);
}

int dev_reserve(const sgp_lattice* L, DevBuf& b, size_t bytes, hipStream_t s) {
  if (b.bytes >= bytes) return SGP_OK;
  if (b.ptr) {
    int rc = wait_last_use(L);
    if (rc) return rc;
    dev_free(b);
  }
  return dev_alloc(b, bytes, s);
}

// ---------------------------------------------------------------------------
// Event profiler.

namespace {
struct ProfRecord {
  int kind;
  hipEvent_t start, stop;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRecord> g_prof_pending;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_prof_pool;
int64_t g_prof_launches[KK_NUM] = {};
double g_prof_ms[KK_NUM] = {};
const char* const kKindNames[KK_NUM] = {
    "fill", "simplex_insert", "count_first", "scan", "compact", "resolve", "neighbors",
    "splat", "splat_gather", "blur", "slice", "cg_init", "cg_scalar", "cg_dir", "cg_alpha", "cg_out", "grad", "sort", "order"};

// Fold completed records into the totals. Caller holds the mutex.
int prof_drain() {
  for (auto& rec : g_prof_pending) {
    hipError_t e = hipEventSynchronize(rec.stop);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize", __FILE__, __LINE__);
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, rec.start, rec.stop);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime", __FILE__, __LINE__);
    g_prof_launches[rec.kind] += 1;
    g_prof_ms[rec.kind] += ms;
    g_prof_pool.emplace_back(rec.start, rec.stop);
  }
  g_prof_pending.clear();
  return SGP_OK;
}
}  // namespace

ProfScope::ProfScope(int kind, hipStream_t s) : stop_(nullptr), stream_(s) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!g_prof_on) return;
  std::pair<hipEvent_t, hipEvent_t> ev;
  if (!g_prof_pool.empty()) {
    ev = g_prof_pool.back();
    g_prof_pool.pop_back();
  } else {
    if (hipEventCreate(&ev.first) != hipSuccess) return;
    if (hipEventCreate(&ev.second) != hipSuccess) {
      (void)hipEventDestroy(ev.first);
      return;
    }
  }
  if (hipEventRecord(ev.first, s) != hipSuccess) {
    g_prof_pool.push_back(ev);
    return;
  }
  g_prof_pending.push_back({kind, ev.first, ev.second});
  stop_ = ev.second;
}

ProfScope::~ProfScope() {
  if (stop_) (void)hipEventRecord(stop_, stream_);
}

// ---------------------------------------------------------------------------
// Host constants: stencil spacing (Section 4.1, eq. balance_coverage) and the
// per-dimension elevation factors (Section 3.2, Splat).

namespace {
const double kPi = 3.14159265358979323846;

double kernel_at(int kernel, double tau) {
  tau = std::fabs(tau);
  if (kernel == SGP_KERNEL_RBF) return std::exp(-0.5 * tau * tau);
  const double a = std::sqrt(3.0);
  return (1.0 + a * tau) * std::exp(-a * tau);
}

// Share of the kernel mass on [-a, a] minus the share of its spectrum on
// [-b, b]; for the Matern-3/2 kernel both integrals are elementary.
double coverage_gap_matern32(double a, double b) {
  const double l3 = std::sqrt(3.0);
  const double spatial = 1.0 - std::exp(-l3 * a) * (1.0 + l3 * a / 2.0);
  const double th = std::atan(b / std::sqrt(3.0));
  const double spectral = (th + 0.5 * std::sin(2.0 * th)) / (kPi / 2.0);
  return spatial - spectral;
}

double spacing_for(int kernel, int r) {
  const int taps = 2 * r + 1;
  // the Gaussian balance erf(s taps / 2 / sqrt2) = erf(pi / s / sqrt2) has root sqrt(2 pi / taps)
  if (kernel == SGP_KERNEL_RBF) return std::sqrt(2.0 * kPi / (double)taps);
  double lo = 1e-3, hi = 1e3;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (coverage_gap_matern32(mid * taps / 2.0, kPi / mid) < 0.0) lo = mid;
    else hi = mid;
  }
  return 0.5 * (lo + hi);
}
}  // namespace

int make_constants(int d, int r, int kernel, const double* ell, double* spacing, double* stencil,
                   double* f) {
  const double s = spacing_for(kernel, r);
  *spacing = s;
  for (int t = -r; t <= r; ++t) stencil[t + r] = kernel_at(kernel, t * s);
  // elevation: column j of the triangular basis has norm sqrt(j(j+1)); one
  // lattice step (length sqrt(d(d+1))) spans s lengthscales
  const double alpha = std::sqrt((double)(d * (d + 1))) / s;
  for (int j = 1; j <= d; ++j) f[j - 1] = alpha / (ell[j - 1] * std::sqrt((double)(j * (j + 1))));
  return SGP_OK;
}

// ---------------------------------------------------------------------------

__global__ void k_fill_u32(uint32_t* __restrict__ p, size_t count, uint32_t value) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = value;
}

int launch_fill_u32(uint32_t* p, size_t count, uint32_t value, hipStream_t s) {
  if (count == 0) return SGP_OK;
  size_t blocks = (count + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
  ProfScope ps(KK_FILL, s);
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(kBlock), 0, s, p, count, value);
  SGP_LAUNCH_CHECK("k_fill_u32");
  return SGP_OK;
}

}  // namespace sgp

using namespace sgp;

namespace sgp {
namespace {
std::atomic<int> g_cg_graph{1};
std::atomic<int> g_blur_fuse{1};
std::atomic<int> g_cg_fuse{1};
}
bool profiling() {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  return g_prof_on;
}
bool cg_graphs_enabled() { return g_cg_graph.load() != 0; }
bool blur_fuse_enabled() { return g_blur_fuse.load() != 0; }
std::atomic<int64_t>& blur_seq_threshold() {
  static std::atomic<int64_t> t{tuning().blur_seq_mib > 0 ? (int64_t)tuning().blur_seq_mib << 20 : -1};
  return t;
}
bool blur_seq_for(double bytes) {
  const int64_t t = blur_seq_threshold().load();
  return t >= 0 && bytes > (double)t;
}
bool cg_fuse_enabled() { return g_cg_fuse.load() != 0; }
hipStream_t capture_stream() {
  constexpr int kMaxDevices = 64;
  thread_local hipStream_t streams[kMaxDevices] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess)
    streams[dev] = nullptr;
  return streams[dev];
}
}  // namespace sgp

extern "C" {

void sgp_opts_default(sgp_opts* o) {
  if (!o) return;
  o->order = 1;
  o->kernel = SGP_KERNEL_RBF;
  o->blur = SGP_BLUR_SYMMETRIC;
  o->outputscale = 1.0f;
  o->load_factor = 0.0f;  // automatic: the autotuned table shape, else 0.5
  o->solve_rows = 0;
}

const char* sgp_last_error(void) { return g_err; }

int sgp_set_allocator(void* (*alloc)(size_t bytes, void* stream), void (*free_fn)(void* ptr, void* stream)) {
  using namespace sgp;
  if ((alloc == nullptr) != (free_fn == nullptr)) {
    set_error("sgp_set_allocator: give both functions, or neither for the built-in pool");
    return SGP_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  if (g_live != 0) {
    set_error("sgp_set_allocator: %lld device blocks of the current allocator are still held; "
              "free every lattice first", (long long)g_live);
    return SGP_EINVAL;
  }
  if (alloc && !g_user_alloc) flush_block_caches();  // idle pool blocks stay with the pool
  g_user_alloc = alloc;
  g_user_free = free_fn;
  return SGP_OK;
}

int lattice_info(const sgp_lattice* L, int64_t* n, int32_t* d, int64_t* m, int64_t* device_bytes) {
  if (!L) {
    set_error("lattice_info: NULL lattice");
    return SGP_EINVAL;
  }
  if (n) *n = L->n;
  if (d) *d = L->d;
  if (m) *m = L->m;
  if (device_bytes)
    *device_bytes = (int64_t)(L->perm.bytes + L->loc.bytes + L->ws.bytes + L->tile_off.bytes + L->stile_off.bytes +
                              L->tile_verts.bytes + L->run_rel.bytes + L->ent_lp.bytes + L->ent_w.bytes +
                              L->occ_ptr.bytes + L->run_dst.bytes + L->row_vert.bytes + L->nbr.bytes + L->int2can.bytes +
                              L->keys.bytes + L->ubuf.bytes + L->cgvec.bytes + L->cgred.bytes);
  return SGP_OK;
}

int lattice_export(const sgp_lattice* L, int32_t* keys, int32_t* idx, float* w, int32_t* nbr) {
  if (!L) {
    set_error("lattice_export: NULL lattice");
    return SGP_EINVAL;
  }
  SGP_HIP(hipSetDevice(L->device));
  int rc0 = wait_last_use(L);
  if (rc0) return rc0;
  const int D = L->d + 1, T = 2 * L->order;
  const int64_t n = L->n, m = L->m;
  if (keys) SGP_HIP(hipMemcpy(keys, L->keys.ptr, sizeof(int32_t) * m * L->d, hipMemcpyDeviceToHost));
  std::vector<int32_t> int2can;
  if (idx || nbr) {
    int2can.resize(m);
    SGP_HIP(hipMemcpy(int2can.data(), L->int2can.ptr, sizeof(int32_t) * m, hipMemcpyDeviceToHost));
  }
  if (idx || w) {
    // internal (sorted point, tile run) -> caller's point order, canonical vertex
    const int P = L->tile_points;
    std::vector<uint32_t> perm(n);
    std::vector<uint16_t> loc((size_t)n * D);
    std::vector<float> ws((size_t)n * D);
    std::vector<int32_t> toff(L->ntiles + 1), tverts(L->nrun);
    SGP_HIP(hipMemcpy(perm.data(), L->perm.ptr, sizeof(uint32_t) * n, hipMemcpyDeviceToHost));
    SGP_HIP(hipMemcpy(loc.data(), L->loc.ptr, sizeof(uint16_t) * n * D, hipMemcpyDeviceToHost));
    SGP_HIP(hipMemcpy(ws.data(), L->ws.ptr, sizeof(float) * n * D, hipMemcpyDeviceToHost));
    SGP_HIP(hipMemcpy(toff.data(), L->tile_off.ptr, sizeof(int32_t) * toff.size(), hipMemcpyDeviceToHost));
    SGP_HIP(hipMemcpy(tverts.data(), L->tile_verts.ptr, sizeof(int32_t) * tverts.size(),
                      hipMemcpyDeviceToHost));
    for (int64_t ip = 0; ip < n; ++ip) {
      const int64_t i = perm[ip];
      const int32_t base = toff[ip / P];
      for (int k = 0; k < D; ++k) {
        if (idx) idx[i * D + k] = int2can[tverts[base + loc[ip * D + k]]];
        if (w) w[i * D + k] = ws[ip * D + k];
      }
    }
  }
  if (nbr) {
    // device layout [direction][internal point][offset] -> [canonical point][direction][offset]
    std::vector<int32_t> tmp((size_t)D * T * m);
    SGP_HIP(hipMemcpy(tmp.data(), L->nbr.ptr, sizeof(int32_t) * tmp.size(), hipMemcpyDeviceToHost));
    for (int k = 0; k < D; ++k)
      for (int64_t ji = 0; ji < m; ++ji)
        for (int t = 0; t < T; ++t) {
          const int32_t v = tmp[((size_t)k * m + ji) * T + t];
          nbr[((size_t)int2can[ji] * D + k) * T + t] = v >= 0 ? int2can[v] : -1;
        }
  }
  return SGP_OK;
}

void lattice_free(sgp_lattice* L) {
  if (!L) return;
  (void)hipSetDevice(L->device);
  // wait for the last use without replacing the thread's error message: a
  // failed build frees its lattice on the way out and reports its own error
  if (L->last_use) (void)hipEventSynchronize(L->last_use);
  for (DevBuf* b : {&L->perm, &L->loc, &L->ws, &L->tile_off, &L->stile_off, &L->tile_verts, &L->run_rel,
                   &L->ent_lp, &L->ent_w, &L->occ_ptr, &L->run_dst, &L->row_vert, &L->nbr, &L->int2can, &L->keys})
    dev_free(*b);
  dev_free(L->ubuf);
  dev_free(L->cgvec);
  dev_free(L->cgred);
  if (L->last_use) (void)hipEventDestroy(L->last_use);
  delete L;
}


int sgp_cache_info(int64_t* bytes, int32_t* blocks) {
  sgp::idle_cache_info(bytes, blocks);
  return SGP_OK;
}

int sgp_debug_inject_oom(int32_t count) {
  sgp::inject_oom(count);
  return SGP_OK;
}

int sgp_cg_graph_enable(int on) { return g_cg_graph.exchange(on != 0 ? 1 : 0); }
int sgp_cg_fuse_enable(int on) { return g_cg_fuse.exchange(on != 0 ? 1 : 0); }
int sgp_blur_fuse_enable(int on) { return g_blur_fuse.exchange(on != 0 ? 1 : 0); }
int64_t sgp_blur_seq_bytes(int64_t bytes) { return blur_seq_threshold().exchange(bytes < 0 ? -1 : bytes); }

int sgp_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
  return SGP_OK;
}

int sgp_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  int rc = prof_drain();
  for (int k = 0; k < KK_NUM; ++k) {
    g_prof_launches[k] = 0;
    g_prof_ms[k] = 0.0;
  }
  return rc;
}

int sgp_profile_kinds(void) { return KK_NUM; }

const char* sgp_profile_name(int kind) {
  return (kind >= 0 && kind < KK_NUM) ? kKindNames[kind] : "";
}

int sgp_profile_read(int kind, int64_t* launches, double* total_ms) {
  if (kind < 0 || kind >= KK_NUM) {
    set_error("sgp_profile_read: kind %d out of range", kind);
    return SGP_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_prof_mu);
  int rc = prof_drain();
  if (launches) *launches = g_prof_launches[kind];
  if (total_ms) *total_ms = g_prof_ms[kind];
  return rc;
}

}  // extern "C"
