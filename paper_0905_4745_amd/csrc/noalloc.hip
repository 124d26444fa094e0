// Device workspace of the allocation-free entry point (srft_sketch_noalloc):
// a file-scope device array of kNoAllocBytes, one copy per GPU, held until
// the process ends.  Host code never uses the array's name as an address:
// its device address is looked up once per device (noalloc_init, called by
// mn_create with that device current) and kept; the entry point hands
// offsets of that address to its kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.hpp"

namespace mn {

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
// what the twiddle region of each device's array holds: (N << 1) | single,
// or -1 (nothing yet)
int64_t g_tag[kMaxDevices];
bool g_tag_init = false;
}  // namespace

hipError_t noalloc_init(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  if (!g_tag_init) {
    for (auto& t : g_tag) t = -1;
    g_tag_init = true;
  }
  if (g_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (p == nullptr) return hipErrorInvalidSymbol;
  g_ptr[device] = p;
  g_tag[device] = -1;
  return hipSuccess;
}

void* noalloc_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  return (device >= 0 && device < kMaxDevices) ? g_ptr[device] : nullptr;
}

bool noalloc_twiddle_swap(int device, int64_t tag) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (device < 0 || device >= kMaxDevices) return true;
  const bool stale = g_tag[device] != tag;
  g_tag[device] = tag;
  return stale;
}

}  // namespace mn
