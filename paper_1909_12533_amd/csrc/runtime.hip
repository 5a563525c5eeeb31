// Device memory and stream runtime of the library: a per-context caching
// allocator (optionally over a caller-supplied allocator, e.g. PyTorch's
// caching allocator), and stream-ordered host<->device transfers.
#include "internal.h"

namespace sp2 {

Buf &Buf::operator=(Buf &&o) noexcept {
  if (this != &o) {
    reset();
    ctx = o.ctx;
    p = o.p;
    bytes = o.bytes;
    o.ctx = nullptr;
    o.p = nullptr;
    o.bytes = 0;
  }
  return *this;
}

void Buf::reset() {
  if (ctx && p) ctx->release(p, bytes);
  ctx = nullptr;
  p = nullptr;
  bytes = 0;
}

void *Ctx::raw_alloc(size_t bytes) {
  void *p = nullptr;
  if (ualloc) {
    p = ualloc(bytes, uuser);
  } else {
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
  }
  return p;
}

void Ctx::raw_free(void *p) {
  if (!p) return;
  if (ufree)
    ufree(p, uuser);
  else
    (void)hipFree(p);
}

static size_t round_bytes(size_t b) {
  const size_t a = 256;
  if (b == 0) b = a;
  return (b + a - 1) / a * a;
}

Buf Ctx::alloc(size_t bytes) {
  bytes = round_bytes(bytes);
  Buf b;
  auto it = cache.lower_bound(bytes);
  if (it != cache.end() && it->first <= bytes + bytes / 4) {
    b.p = it->second;
    b.bytes = it->first;
    cached_bytes -= it->first;
    cache.erase(it);
  } else {
    void *p = raw_alloc(bytes);
    if (!p) {
      sync();
      trim();
      p = raw_alloc(bytes);
    }
    if (!p) {
      size_t fr = 0, tot = 0;
      (void)hipMemGetInfo(&fr, &tot);
      fail(SP2_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed (library live " +
                            std::to_string(live_bytes) + " bytes, device free " + std::to_string(fr) + " of " +
                            std::to_string(tot) + ")");
    }
    b.p = p;
    b.bytes = bytes;
  }
  b.ctx = this;
  live_bytes += b.bytes;
  if (live_bytes > peak_bytes) peak_bytes = live_bytes;
  return b;
}

// Buffers up to 64 MB are kept for reuse (the many small pattern, map and
// reduction arrays of every iteration); larger ones go straight back to the
// allocator, which can split and merge them (matrix pools are tens of GB at
// the largest workloads, and holding them here would strand that memory).
void Ctx::release(void *p, size_t bytes) {
  live_bytes -= bytes;
  if (bytes > ((size_t)64 << 20)) {
    raw_free(p);
    return;
  }
  cache.emplace(bytes, p);
  cached_bytes += bytes;
}

void Ctx::trim() {
  if (!cache.empty()) (void)hipStreamSynchronize(stream);
  for (auto &kv : cache) raw_free(kv.second);
  cache.clear();
  cached_bytes = 0;
}

void Ctx::sync() { SP2_HIP(hipStreamSynchronize(stream)); }

void Ctx::d2h(void *dst, const void *src, size_t bytes) {
  if (bytes == 0) return;
  SP2_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, stream));
  SP2_HIP(hipStreamSynchronize(stream));
}

void Ctx::h2d(void *dst, const void *src, size_t bytes) {
  if (bytes == 0) return;
  SP2_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream));
  SP2_HIP(hipStreamSynchronize(stream));
}

}  // namespace sp2
