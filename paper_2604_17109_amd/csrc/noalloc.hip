// pim_energy_noalloc: the binary64 energy evaluation of pim_energy without
// any device allocation, for callers that cannot allocate device memory.
//
// pim_energy stages the configurations and the energies in device memory it
// allocates per call.  This variant stages them in `scratch`, a fixed
// file-scope device array of PIM_NOALLOC_SCRATCH_BYTES bytes, which every GPU
// the library runs on holds until the process ends.  In host code the name
// `scratch` is only a host-side stand-in: its device address is looked up
// once per device with hipGetSymbolAddress (with that device current) and
// only that address is ever handed to kernels and copies.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "internal.hpp"

namespace {

static __device__ __align__(256) unsigned char scratch[PIM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up on the
// first call on that device).
pim_status device_scratch(unsigned char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return pim::fail(PIM_ERR_DEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return pim::fail(PIM_ERR_UNSUPPORTED, "device %d outside the %d the library tracks", dev, kMaxDevices);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return pim::fail(PIM_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch[dev];
  return PIM_OK;
}

}  // namespace

extern "C" pim_status pim_energy_noalloc(const pim_instance* inst, const int8_t* spins, int32_t count, double* out,
                                         void* stream) {
  using pim::fail;
  try {
    if (!inst || !spins || !out) return fail(PIM_ERR_INVALID, "NULL argument");
    if (count < 1) return fail(PIM_ERR_INVALID, "count must be >= 1");
    const int n = inst->rule.n;
    bool on_device = false;
    {
      hipPointerAttribute_t attr{};
      if (hipPointerGetAttributes(&attr, spins) == hipSuccess)
        on_device = attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
      else
        (void)hipGetLastError();  // an unknown pointer is host memory, not an error
    }
    // scratch layout: the energies (256-byte aligned), then the staged spins
    const size_t e_bytes = ((size_t)count * sizeof(double) + 255) & ~(size_t)255;
    const size_t s_bytes = on_device ? 0 : (size_t)count * n;
    if (e_bytes + s_bytes > (size_t)PIM_NOALLOC_SCRATCH_BYTES)
      return fail(PIM_ERR_INVALID, "%d configurations of %d spins need %zu bytes, more than the %d-byte scratch",
                  count, n, e_bytes + s_bytes, PIM_NOALLOC_SCRATCH_BYTES);
    if (!on_device)
      for (size_t i = 0; i < s_bytes; ++i)
        if (spins[i] != 1 && spins[i] != -1)
          return fail(PIM_ERR_INVALID, "spin value %d at %zu is not +-1", (int)spins[i], i);
    unsigned char* base = nullptr;
    pim_status st = device_scratch(&base);
    if (st != PIM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    double* d_out = reinterpret_cast<double*>(base);
    int8_t* d_spins = on_device ? nullptr : reinterpret_cast<int8_t*>(base + e_bytes);
    pim::EnergyArgs ea{};
    ea.jf32 = inst->d_jf32;
    ea.h = (!inst->rule.real && inst->has_h) ? inst->d_h : nullptr;
    ea.jf64 = inst->rule.real ? inst->d_j64 : nullptr;
    ea.hf64 = (inst->rule.real && inst->has_h) ? inst->d_h64 : nullptr;
    ea.spins = on_device ? spins : d_spins;
    ea.out = d_out;
    ea.n = n;
    ea.jstride = inst->jstride;
    ea.stride = n;
    ea.count = count;
    hipError_t e = on_device ? hipSuccess : hipMemcpyAsync(d_spins, spins, s_bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = pim::launch_energy_f64(ea, s);
    if (e == hipSuccess) e = hipMemcpyAsync(out, d_out, (size_t)count * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    else (void)hipStreamSynchronize(s);  // a queued copy may still read the caller's spins
    if (e != hipSuccess) return fail(PIM_ERR_DEVICE, "pim_energy_noalloc failed: %s", hipGetErrorString(e));
    return PIM_OK;
  } catch (...) {
    return fail(PIM_ERR_INVALID, "internal error in pim_energy_noalloc");
  }
}
