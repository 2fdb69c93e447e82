// Launchers of the host side (own translation unit): the functor id and dtype
// select the same concrete types as on the device, then host threads run them.
#include "hdc_host_side.hpp"

namespace hdc {

hdc_status run_host_map(const hdc_functor& f, hdc_dtype dt, const void* x, void* y, int64_t n, int32_t nthreads) {
  if (dt == HDC_I32)
    return with_int_fn(f, [&](auto fn) {
      host_map<decltype(fn), I32>(fn, x, y, n, nthreads);
      return HDC_OK;
    });
  return with_float_storage(dt, [&](auto s) {
    using S = decltype(s);
    return with_float_fn(f, [&](auto fn) -> hdc_status {
      using F = decltype(fn);
      if constexpr (F::binary) {
        return fail(HDC_ERR_UNSUPPORTED, "PRODUCT cannot be mapped");
      } else {
        host_map<F, S>(fn, x, y, n, nthreads);
        return HDC_OK;
      }
    });
  });
}

hdc_status run_host_reduce(const hdc_functor& f, hdc_dtype dt, const void* x, const void* z, int64_t n,
                           hdc_accum acc, void* out, int32_t nthreads) {
  if (dt == HDC_I32)
    return with_int_fn(f, [&](auto fn) {
      host_reduce<decltype(fn), I32, IntAcc>(fn, x, z, n, out, nthreads);
      return HDC_OK;
    });
  return with_float_storage(dt, [&](auto s) {
    using S = decltype(s);
    return with_float_fn(f, [&](auto fn) -> hdc_status {
      using F = decltype(fn);
      if (acc == HDC_ACC_COMPENSATED)
        host_reduce<F, S, CompAcc>(fn, x, z, n, out, nthreads);
      else
        host_reduce<F, S, PlainAcc>(fn, x, z, n, out, nthreads);
      return HDC_OK;
    });
  });
}

}  // namespace hdc
