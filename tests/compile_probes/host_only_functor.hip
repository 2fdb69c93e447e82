// Compile probe: a callable without a device-capable tag must not instantiate
// a kernel (a stray call is a compile error, as the paper's section 2.1 goal).
#include "hdc_kernels.hpp"

struct HostOnly {  // no `hdc` member: the trait reads it as host-only
  static constexpr bool binary = false;
  float operator()(float x) const { return x + 1.0f; }
};

#ifdef PROBE_DEVICE_TAGGED
struct Tagged {
  static constexpr hdc::HDC hdc = hdc::HDC::HstDev;
  static constexpr bool binary = false;
  __host__ __device__ float operator()(float x) const { return x + 1.0f; }
};
using Callable = Tagged;
#else
using Callable = HostOnly;
#endif

static_assert(hdc::hdc_of<HostOnly> == hdc::HDC::Hst);
static_assert(hdc::hdc_of<hdc::Horner> == hdc::HDC::HstDev);

void launch(const float* x, float* y, hdc::Range r) {
  hdc::map_kernel<Callable, hdc::F32, 1, true><<<1, 64>>>(Callable{}, x, y, r);
}

#ifdef PROBE_HOST_SIDE
#include "hdc_host_side.hpp"
struct DevOnly {  // device-only callable: the host side must reject it
  static constexpr hdc::HDC hdc = hdc::HDC::Dev;
  static constexpr bool binary = false;
  __device__ float operator()(float x) const { return x; }
};
#ifdef PROBE_HOST_DEVONLY
using HostCallable = DevOnly;
#else
using HostCallable = hdc::Horner;
#endif
void host_probe(const float* x, float* y) { hdc::host_map<HostCallable, hdc::F32>(HostCallable{}, x, y, 4, 1); }
#endif
