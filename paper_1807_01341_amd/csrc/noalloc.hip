// One whole step for callers that cannot allocate device memory: the step
// of sph_step on a transient context whose every device buffer is carved
// from a fixed array of this library (a bump allocator over `scratch`), and
// whose small device-to-host reads are copies into host memory of the
// context object (no page-locked allocation).
#include <stdio.h>

#include <mutex>

#include "sph_internal.h"

// Bytes of the static scratch array and the largest particle count a call
// accepts (a step of that many particles, clustered, uses well under the
// array: the buffers of a context scale with the particle count, and the
// bump allocator also keeps the blocks a buffer outgrows).
#define SPH_NOALLOC_SCRATCH_BYTES (256ull << 20)
#define SPH_NOALLOC_MAX_N ((int64_t)1 << 18)

static __device__ __align__(256) unsigned char scratch[SPH_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {nullptr};

// The device address of this device's copy of `scratch` (the array's name in
// host code is only a handle for HIP_SYMBOL): looked up once per device,
// with that device current.
hipError_t scratch_on_current_device(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

struct Arena {
  char *base = nullptr;
  size_t cap = 0, used = 0, peak = 0;
  bool exhausted = false;
};

void *arena_alloc(size_t bytes, void *, void *user) {
  Arena *a = static_cast<Arena *>(user);
  const size_t b = (bytes + 255) & ~(size_t)255;
  if (b > a->cap - a->used) {
    a->exhausted = true;
    return nullptr;
  }
  void *p = a->base + a->used;
  a->used += b;
  if (a->used > a->peak) a->peak = a->used;
  return p;
}

void arena_free(void *, void *, void *) {}

void put_error(char *err, size_t cap, const char *msg) {
  if (!err || cap == 0) return;
  size_t k = 0;
  for (; msg && msg[k] && k + 1 < cap; ++k) err[k] = msg[k];
  err[k] = 0;
}

}  // namespace

extern "C" sph_status sph_step_noalloc(const sph_params *p, void *hip_stream, sph_particles *parts, int64_t n,
                                       int64_t *perm_out, int max_active_bin, int64_t *n_active_host,
                                       int entropy_from_u, int64_t ti, double t_min, int64_t drift_int,
                                       int first_step, int64_t *scratch_used_host, char *err, size_t err_cap) {
  put_error(err, err_cap, "");
  if (!p || !parts) {
    put_error(err, err_cap, "step_noalloc: null parameters or particles");
    return SPH_EINVAL;
  }
  if (n <= 0 || n > SPH_NOALLOC_MAX_N) {
    char msg[160];
    snprintf(msg, sizeof msg, "step_noalloc: n = %lld outside [1, %lld], the limit of the static scratch array",
             (long long)n, (long long)SPH_NOALLOC_MAX_N);
    put_error(err, err_cap, msg);
    return SPH_EINVAL;
  }
  void *base = nullptr;
  const hipError_t e = scratch_on_current_device(&base);
  if (e != hipSuccess) {
    put_error(err, err_cap, "step_noalloc: the static scratch array has no device address");
    return SPH_EDEVICE;
  }
  Arena arena;
  arena.base = static_cast<char *>(base);
  arena.cap = SPH_NOALLOC_SCRATCH_BYTES;
  sph_ctx *ctx = new (std::nothrow) sph_ctx();
  if (!ctx) {
    put_error(err, err_cap, "step_noalloc: no host memory for the context");
    return SPH_ENOMEM;
  }
  sph_status st = ctx_init(ctx, p, hip_stream, arena_alloc, arena_free, &arena, false);
  if (st == SPH_OK) st = sph_step(ctx, parts, n, perm_out, max_active_bin, n_active_host, entropy_from_u, ti, t_min,
                                  drift_int, first_step);
  // the context is gone when this call returns, and the next call reuses the array
  const sph_status st_sync = sph_sync(ctx);
  if (st == SPH_OK) st = st_sync;
  if (st != SPH_OK) {
    if (st == SPH_ENOMEM && arena.exhausted)
      put_error(err, err_cap, "step_noalloc: the static scratch array is exhausted");
    else
      put_error(err, err_cap, ctx->err.c_str());
  }
  if (scratch_used_host) *scratch_used_host = (int64_t)arena.peak;
  sph_destroy(ctx);
  return st;
}
