// Device memory and stream runtime of the library: a per-context caching
// allocator (optionally over a caller-supplied allocator, e.g. PyTorch's
// caching allocator), and stream-ordered host<->device transfers.
#include <chrono>

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
  const auto t0 = std::chrono::steady_clock::now();
  struct Timer {
    Ctx *c;
    std::chrono::steady_clock::time_point t0;
    ~Timer() {
      c->raw_alloc_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      c->n_raw_alloc++;
    }
  } timer{this, t0};
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
  const auto t0 = std::chrono::steady_clock::now();
  struct Timer {
    Ctx *c;
    std::chrono::steady_clock::time_point t0;
    ~Timer() {
      c->raw_free_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      c->n_raw_free++;
    }
  } timer{this, t0};
  if (ufree)
    ufree(p, uuser);
  else
    (void)hipFree(p);
}

// Small buffers are rounded to 256 bytes.  Large ones (matrix pools, BF16x3
// images, the correction's intermediates: hundreds of MB to tens of GB, a
// slightly different size at every iteration) are rounded up to one of 16
// steps per power of two (at most 6.25% more), so that the buffer released by
// one iteration serves the next one's request of about the same size.
static size_t round_bytes(size_t b) {
  const size_t a = 256;
  if (b == 0) b = a;
  b = (b + a - 1) / a * a;
  if (b > BIG_BUFFER) {
    size_t p2 = (size_t)1 << (63 - __builtin_clzll((unsigned long long)b));
    const size_t step = p2 / 16;
    b = (b + step - 1) / step * step;
  }
  return b;
}

Buf Ctx::alloc(size_t bytes) {
  bytes = round_bytes(bytes);
  Buf b;
  auto it = cache.lower_bound(bytes);
  const size_t slack = bytes > BIG_BUFFER ? bytes / 8 : bytes / 4;
  if (it != cache.end() && it->first <= bytes + slack) {
    b.p = it->second;
    b.bytes = it->first;
    cached_bytes -= it->first;
    cache.erase(it);
  } else {
    // the runtime allocates its own memory at kernel launch (the private
    // memory of kernels with register spills): keep free device memory above
    // a reserve by releasing cached buffers before a new large allocation
    if (bytes > BIG_BUFFER && cached_bytes > 0) {
      size_t fr = 0, tot = 0;
      if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        (void)hipGetLastError();
      } else if (fr < bytes + FREE_RESERVE) {
        sync();
        trim();
      }
    }
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

// Released buffers are kept for reuse by later requests of the same rounded
// size on this stream: the many small pattern, map and reduction arrays of
// every iteration, and the large pools, whose allocation and release through
// the device allocator cost about a second per 100 GB.  A request the device
// cannot serve first releases the whole cache and tries again (alloc), and
// callers release it between calls (sp2_trim).
void Ctx::release(void *p, size_t bytes) {
  live_bytes -= bytes;
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

hipStream_t Ctx::copies() {
  if (!copy_stream) SP2_HIP(hipStreamCreateWithFlags(&copy_stream, hipStreamNonBlocking));
  return copy_stream;
}

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
