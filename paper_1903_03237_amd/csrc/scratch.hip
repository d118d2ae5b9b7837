// The workspace of contexts made by fmnmf_init_noalloc: a file-scope device
// array per GPU, held from the library's first use on that GPU until the
// process ends.  Host code never uses the array's name as an address: its
// device address is looked up once per device, with that device current,
// and kept in `g_slots`.
#include <mutex>
#include <vector>

#include "../../include/fmnmf.h"
#include "scratch.h"

namespace fmnmf {

static __device__ __align__(256) unsigned char scratch[FMNMF_SCRATCH_BYTES];

namespace {
struct Slot {
  void* ptr = nullptr;  // device address of `scratch` on this device
  bool in_use = false;  // held by a live context
};
std::mutex g_mu;
std::vector<Slot> g_slots;  // indexed by device ordinal
}  // namespace

int scratch_acquire(int dev, void** ptr, hipError_t* err) {
  std::lock_guard<std::mutex> lk(g_mu);
  if ((int)g_slots.size() <= dev) g_slots.resize(dev + 1);
  Slot& s = g_slots[dev];
  if (!s.ptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
      return SCRATCH_HIP_ERROR;
    }
    s.ptr = p;
  }
  if (s.in_use) return SCRATCH_IN_USE;
  s.in_use = true;
  *ptr = s.ptr;
  return SCRATCH_OK;
}

void scratch_release(int dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (dev >= 0 && dev < (int)g_slots.size()) g_slots[dev].in_use = false;
}

}  // namespace fmnmf
