// Context plumbing: device memory through the optional caller allocator,
// named scratch, kernel profiling with hipEvents on the context's stream.
#include <algorithm>

#include "common.hpp"

namespace pts {

DevMem::~DevMem() { reset(); }

void DevMem::reset() {
  if (ptr && ctx) ctx->dfree(ptr, bytes);
  ptr = nullptr;
  bytes = 0;
}

void* DevMem::ensure(Ctx* c, size_t nbytes) {
  if (nbytes == 0) nbytes = 1;
  if (ptr && bytes >= nbytes) return ptr;
  reset();
  ctx = c;
  // grow geometrically to avoid repeated reallocation
  size_t want = std::max(nbytes, (size_t)256);
  ptr = c->dalloc(want);
  bytes = want;
  return ptr;
}

void* Ctx::dalloc(size_t bytes) {
  void* p = nullptr;
  if (has_alloc) {
    p = alloc.alloc(alloc.user, bytes, (void*)stream);
    if (!p) fail(PTS_ERR_OOM, "caller allocator refused " + std::to_string(bytes) + " bytes");
    return p;
  }
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(e == hipErrorOutOfMemory ? PTS_ERR_OOM : PTS_ERR_HIP,
         "hipMalloc(" + std::to_string(bytes) + "): " + hipGetErrorString(e));
  }
  return p;
}

void Ctx::dfree(void* p, size_t bytes) {
  if (!p) return;
  if (has_alloc) {
    alloc.release(alloc.user, p, bytes, (void*)stream);
    return;
  }
  // memory may still be in use by queued work on the stream
  (void)hipStreamSynchronize(stream);
  (void)hipFree(p);
}

void Ctx::prof_begin(const char* name) {
  hipEvent_t a, b;
  if (prof_free.size() >= 2) {
    a = prof_free.back();
    prof_free.pop_back();
    b = prof_free.back();
    prof_free.pop_back();
  } else {
    PTS_HIP(hipEventCreate(&a));
    PTS_HIP(hipEventCreate(&b));
  }
  PTS_HIP(hipEventRecord(a, stream));
  prof_pending.push_back({std::string(name), {a, b}});
}

void Ctx::prof_end() {
  // runs in a destructor: never throws
  if (prof_pending.empty()) return;
  (void)hipEventRecord(prof_pending.back().second.second, stream);
  if (prof_pending.size() >= 2048) {
    try {
      prof_drain();
    } catch (...) {
    }
  }
}

void Ctx::prof_drain() {
  if (prof_pending.empty()) return;
  PTS_HIP(hipStreamSynchronize(stream));
  for (auto& p : prof_pending) {
    float ms = 0.f;
    PTS_HIP(hipEventElapsedTime(&ms, p.second.first, p.second.second));
    auto it = prof_table.find(p.first);
    if (it == prof_table.end()) {
      prof_order.push_back(p.first);
      it = prof_table.emplace(p.first, ProfEntry{}).first;
    }
    it->second.total_ms += ms;
    it->second.launches += 1;
    prof_free.push_back(p.second.first);
    prof_free.push_back(p.second.second);
  }
  prof_pending.clear();
}

Ctx::~Ctx() {
  (void)hipStreamSynchronize(stream);
  for (auto& p : prof_pending) {
    (void)hipEventDestroy(p.second.first);
    (void)hipEventDestroy(p.second.second);
  }
  for (auto e : prof_free) (void)hipEventDestroy(e);
}

}  // namespace pts
