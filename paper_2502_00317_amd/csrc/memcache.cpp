// Block cache for the library's device and pinned host memory.
//
// hipFree and hipHostFree wait for the whole device, so a free issued while
// another stream runs a long search stalls the caller until that search
// ends.  The serving path frees graphs and grows workspaces while other
// streams are busy; it must never wait for them.  Freed blocks therefore go
// back to a per-device cache and are handed out again for requests of a
// similar size; only blocks beyond the cache's byte cap, and dist_mem_trim,
// give memory back to the runtime.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <unordered_map>

#include "internal.h"

namespace {

constexpr size_t kDevCap = (size_t)16 << 30;    // cached device bytes per device
constexpr size_t kHostCap = (size_t)1 << 30;    // cached pinned bytes per kind

size_t round_size(size_t b) {
  if (b < 16) b = 16;
  if (b <= ((size_t)4 << 20)) return (b + 511) & ~(size_t)511;
  return (b + ((size_t)2 << 20) - 1) & ~(((size_t)2 << 20) - 1);
}

struct Pool {
  std::multimap<size_t, void*> free_blocks;  // size -> block
  size_t cached = 0;
};

struct Block {
  size_t size;
  int key;  // device id, or -1 - flags for pinned host memory
};

std::mutex g_mu;
std::map<int, Pool> g_pools;
std::unordered_map<void*, Block> g_live;  // every block the cache handed out or holds

// a cached block of at least `need` bytes and not much larger, or nullptr
void* take(Pool& P, size_t need) {
  auto it = P.free_blocks.lower_bound(need);
  if (it == P.free_blocks.end() || it->first > 2 * need + ((size_t)1 << 20)) return nullptr;
  void* p = it->second;
  P.cached -= it->first;
  P.free_blocks.erase(it);
  return p;
}

}  // namespace

int dev_alloc(void** p, size_t bytes) {
  *p = nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DIST_E_DEVICE;
  const size_t need = round_size(bytes);
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (void* q = take(g_pools[dev], need)) {
      *p = q;
      return DIST_OK;
    }
  }
  void* q = nullptr;
  if (hipMalloc(&q, need) != hipSuccess) {
    // the cache may hold enough memory: give it back and try once more
    dist_mem_trim();
    if (hipMalloc(&q, need) != hipSuccess) return DIST_E_NOMEM;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  g_live[q] = Block{need, dev};
  *p = q;
  return DIST_OK;
}

void dev_free(void* p) {
  if (!p) return;
  int key = 0;  // blocks the cache did not hand out are device blocks
  {
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_live.find(p);
    if (it != g_live.end()) {
      key = it->second.key;
      Pool& P = g_pools[key];
      const size_t cap = key >= 0 ? kDevCap : kHostCap;
      if (P.cached + it->second.size <= cap) {
        P.free_blocks.emplace(it->second.size, p);
        P.cached += it->second.size;
        return;
      }
      g_live.erase(it);  // over the cap: back to the runtime
    }
  }
  if (key >= 0)
    (void)hipFree(p);
  else
    (void)hipHostFree(p);
}

int pinned_alloc(void** p, size_t bytes, unsigned flags) {
  *p = nullptr;
  const size_t need = round_size(bytes);
  const int key = -1 - (int)flags;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (void* q = take(g_pools[key], need)) {
      *p = q;
      return DIST_OK;
    }
  }
  void* q = nullptr;
  if (hipHostMalloc(&q, need, flags) != hipSuccess) return DIST_E_NOMEM;
  std::lock_guard<std::mutex> lock(g_mu);
  g_live[q] = Block{need, key};
  *p = q;
  return DIST_OK;
}

void pinned_free(void* p) { dev_free(p); }

extern "C" int dist_mem_trim(void) {
  std::multimap<size_t, void*> dev_blocks, host_blocks;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    for (auto& kv : g_pools) {
      for (auto& b : kv.second.free_blocks) {
        g_live.erase(b.second);
        (kv.first >= 0 ? dev_blocks : host_blocks).insert(b);
      }
      kv.second.free_blocks.clear();
      kv.second.cached = 0;
    }
  }
  for (auto& b : dev_blocks) (void)hipFree(b.second);
  for (auto& b : host_blocks) (void)hipHostFree(b.second);
  return DIST_OK;
}

extern "C" int dist_mem_cached(int64_t* device_bytes, int64_t* host_bytes) {
  if (!device_bytes || !host_bytes) return DIST_E_INVALID;
  std::lock_guard<std::mutex> lock(g_mu);
  *device_bytes = 0;
  *host_bytes = 0;
  for (auto& kv : g_pools) (kv.first >= 0 ? *device_bytes : *host_bytes) += (int64_t)kv.second.cached;
  return DIST_OK;
}
