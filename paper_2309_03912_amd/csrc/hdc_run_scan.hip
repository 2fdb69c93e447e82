// Launcher of the scan family (own translation unit).
#include "hdc_launch.hpp"

namespace hdc {

hdc_status run_scan(const hdc_functor& f, hdc_dtype dt, const void* x, void* y, int64_t n, hdc_accum acc,
                    int exclusive, void* ws, const Tuning& t, hipStream_t st) {
  const SegSpec none{nullptr, 0};
  if (dt == HDC_I32)
    return with_int_fn(f, [&](auto fn) {
      return launch_scan<decltype(fn), I32, IntAcc>(fn, x, y, n, exclusive, none, ws, t, st);
    });
  return with_float_storage(dt, [&](auto s) {
    using S = decltype(s);
    return with_float_fn(f, [&](auto fn) -> hdc_status {
      using F = decltype(fn);
      if constexpr (F::binary) {
        return fail(HDC_ERR_UNSUPPORTED, "PRODUCT is not a scan term");
      } else {
        if (acc == HDC_ACC_COMPENSATED)
          return launch_scan<F, S, CompAcc>(fn, x, y, n, exclusive, none, ws, t, st);
        return launch_scan<F, S, PlainAcc>(fn, x, y, n, exclusive, none, ws, t, st);
      }
    });
  });
}

}  // namespace hdc
