// Launcher of the segmented family (own translation unit).
#include "hdc_launch.hpp"

namespace hdc {

hdc_status run_segmented(const hdc_functor& f, hdc_dtype dt, const void* x, const int64_t* off, int64_t nseg,
                         hdc_accum acc, void* out, void* ws, size_t ws_bytes, const Tuning& t, hipStream_t st) {
  if (dt == HDC_I32)
    return with_int_fn(f, [&](auto fn) {
      return launch_segmented<decltype(fn), I32, IntAcc>(fn, x, off, nseg, out, ws, ws_bytes, t, st);
    });
  return with_float_storage(dt, [&](auto s) {
    using S = decltype(s);
    return with_float_fn(f, [&](auto fn) -> hdc_status {
      using F = decltype(fn);
      if constexpr (F::binary) {
        return fail(HDC_ERR_UNSUPPORTED, "PRODUCT is not a segmented fold term");
      } else {
        if (acc == HDC_ACC_COMPENSATED)
          return launch_segmented<F, S, CompAcc>(fn, x, off, nseg, out, ws, ws_bytes, t, st);
        return launch_segmented<F, S, PlainAcc>(fn, x, off, nseg, out, ws, ws_bytes, t, st);
      }
    });
  });
}

}  // namespace hdc
