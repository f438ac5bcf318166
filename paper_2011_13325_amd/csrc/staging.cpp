// Pinned double-buffered staging of large setup copies (staging.hpp).
//
// Two pinned chunks of kChunk bytes are allocated with hipHostMalloc on first use and kept for the
// life of the process (they are shared by every device and every hierarchy; a mutex serialises
// the callers).  Copies below kDirect bytes go straight from pageable memory.
#include "staging.hpp"

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>

namespace eamg {
namespace {

constexpr size_t kChunk = size_t(16) << 20;
constexpr size_t kDirect = size_t(2) << 20;

struct Stage {
  std::mutex mu;
  void *buf[2] = {nullptr, nullptr};
};

Stage &stage() {
  static Stage *st = new Stage();   // never destroyed: the pinned chunks live until exit
  return *st;
}

#define EAMG_TRY(x)                \
  do {                             \
    const hipError_t e_ = (x);     \
    if (e_ != hipSuccess) return e_; \
  } while (0)

hipError_t ensure_chunks(Stage &st) {
  for (void *&b : st.buf)
    if (!b) EAMG_TRY(hipHostMalloc(&b, kChunk, hipHostMallocDefault));
  return hipSuccess;
}

struct Events {
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipError_t init() {
    for (hipEvent_t &e : ev) EAMG_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return hipSuccess;
  }
  ~Events() {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

hipError_t h2d(void *dst, const void *src, size_t bytes, hipStream_t s, Stage &st) {
  EAMG_TRY(ensure_chunks(st));
  Events ev;
  EAMG_TRY(ev.init());
  const char *in = static_cast<const char *>(src);
  char *out = static_cast<char *>(dst);
  size_t i = 0;
  for (size_t off = 0; off < bytes; off += kChunk, ++i) {
    const size_t len = std::min(kChunk, bytes - off);
    const int k = int(i & 1);
    if (i >= 2) EAMG_TRY(hipEventSynchronize(ev.ev[k]));   // chunk k's previous DMA is done
    std::memcpy(st.buf[k], in + off, len);
    EAMG_TRY(hipMemcpyAsync(out + off, st.buf[k], len, hipMemcpyHostToDevice, s));
    EAMG_TRY(hipEventRecord(ev.ev[k], s));
  }
  return hipStreamSynchronize(s);
}

hipError_t d2h(void *dst, const void *src, size_t bytes, hipStream_t s, Stage &st) {
  EAMG_TRY(ensure_chunks(st));
  Events ev;
  EAMG_TRY(ev.init());
  const char *in = static_cast<const char *>(src);
  char *out = static_cast<char *>(dst);
  const size_t n = (bytes + kChunk - 1) / kChunk;
  auto issue = [&](size_t i) -> hipError_t {
    const size_t off = i * kChunk, len = std::min(kChunk, bytes - off);
    EAMG_TRY(hipMemcpyAsync(st.buf[i & 1], in + off, len, hipMemcpyDeviceToHost, s));
    return hipEventRecord(ev.ev[i & 1], s);
  };
  EAMG_TRY(issue(0));
  for (size_t i = 0; i < n; ++i) {
    // chunk i + 1 lands in the buffer whose host copy (chunk i - 1) finished last iteration
    if (i + 1 < n) EAMG_TRY(issue(i + 1));
    EAMG_TRY(hipEventSynchronize(ev.ev[i & 1]));
    const size_t off = i * kChunk, len = std::min(kChunk, bytes - off);
    std::memcpy(out + off, st.buf[i & 1], len);
  }
  return hipStreamSynchronize(s);
}

}  // namespace

// On an error the stream is drained before the staging lock is released, so that no copy still
// queued reads or writes a chunk that the next caller refills.
hipError_t copy_h2d_sync(void *dst, const void *src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  if (bytes < kDirect) {
    EAMG_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
    return hipStreamSynchronize(s);
  }
  Stage &st = stage();
  std::lock_guard<std::mutex> lock(st.mu);
  const hipError_t e = h2d(dst, src, bytes, s, st);
  if (e != hipSuccess) (void)hipStreamSynchronize(s);
  return e;
}

hipError_t copy_d2h_sync(void *dst, const void *src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  if (bytes < kDirect) {
    EAMG_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
    return hipStreamSynchronize(s);
  }
  Stage &st = stage();
  std::lock_guard<std::mutex> lock(st.mu);
  const hipError_t e = d2h(dst, src, bytes, s, st);
  if (e != hipSuccess) (void)hipStreamSynchronize(s);
  return e;
}

}  // namespace eamg
