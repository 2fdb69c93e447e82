// Launcher of the map family (own translation unit).
#include "hdc_launch.hpp"

namespace hdc {

hdc_status run_map(const hdc_functor& f, hdc_dtype dt, const void* x, void* y, int64_t n, const Tuning& t,
                   hipStream_t st) {
  if (dt == HDC_I32)
    return with_int_fn(f, [&](auto fn) { return launch_map<decltype(fn), I32>(fn, x, y, n, t, st); });
  return with_float_storage(dt, [&](auto s) {
    using S = decltype(s);
    return with_float_fn(f, [&](auto fn) -> hdc_status {
      using F = decltype(fn);
      if constexpr (F::binary)
        return fail(HDC_ERR_UNSUPPORTED, "PRODUCT cannot be mapped");
      else
        return launch_map<F, S>(fn, x, y, n, t, st);
    });
  });
}

}  // namespace hdc
