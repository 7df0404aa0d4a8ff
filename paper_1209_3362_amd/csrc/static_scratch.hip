// Library-owned device scratch for nfs_structure_function_noalloc.
//
// One file-scope device array holds the whole workspace of the plan that
// entry point builds (ring, row-pass intermediate, sums, tables). Every GPU
// the library runs on keeps its own copy, at its own address, from the
// first use on that GPU until the process ends. In host code `scratch`
// names a host-side stand-in, not device memory: its device address is
// looked up once per device with hipGetSymbolAddress and only that address
// is handed to kernels and copies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "nfs.h"
#include "nfs_host.hpp"
#include "nfs_kernels.hpp"

namespace {

static __device__ __align__(256) unsigned char scratch[NFS_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

}  // namespace

namespace nfs {

hipError_t static_scratch(int device, void** addr) {
  if (!addr) return hipErrorInvalidValue;
  *addr = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    int current = -1;
    hipError_t e = hipGetDevice(&current);
    if (e != hipSuccess) return e;
    if (current != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (current != device) {
      hipError_t r = hipSetDevice(current);
      if (e == hipSuccess) e = r;
    }
    if (e != hipSuccess) return e;
    if (!p || reinterpret_cast<uintptr_t>(p) % kAlign) return hipErrorInvalidSymbol;
    g_scratch_addr[device] = p;
  }
  *addr = g_scratch_addr[device];
  return hipSuccess;
}

}  // namespace nfs
