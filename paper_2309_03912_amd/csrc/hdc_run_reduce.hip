// Launcher of the transform_reduce / dot family (own translation unit).
#include "hdc_launch.hpp"

namespace hdc {

hdc_status run_reduce(const hdc_functor& f, hdc_dtype dt, const void* x, const void* z, int64_t n, hdc_accum acc,
                      void* out, void* ws, uint64_t* ticket, const Tuning& t, hipStream_t st) {
  if (dt == HDC_I32)
    return with_int_fn(f, [&](auto fn) {
      return launch_reduce<decltype(fn), I32, IntAcc>(fn, x, z, n, out, ws, ticket, t, st);
    });
  if (acc == HDC_ACC_EXACT) {  // checked on entry: IDENTITY on F16 or BF16 storage, PRODUCT on F16
    // (the exact bf16 sum and fp16 dot keep their own two launches)
    if (f.id == HDC_FN_PRODUCT) return launch_exact_f16_dot(x, z, n, out, ws, t, st);
    if (dt == HDC_BF16) return launch_exact_bf16(x, n, out, ws, t, st);
    return launch_reduce<Identity, F16, ExactAcc>(Identity{}, x, z, n, out, ws, ticket, t, st);
  }
  return with_float_storage(dt, [&](auto s) {
    using S = decltype(s);
    return with_float_fn(f, [&](auto fn) -> hdc_status {
      using F = decltype(fn);
      if (acc == HDC_ACC_COMPENSATED) return launch_reduce<F, S, CompAcc>(fn, x, z, n, out, ws, ticket, t, st);
      return launch_reduce<F, S, PlainAcc>(fn, x, z, n, out, ws, ticket, t, st);
    });
  });
}

}  // namespace hdc
