// Launcher of the fused map + reduce family for ONE storage type: this file is
// compiled once per storage type (-DHDC_MR_STORAGE=F32|F16|BF16|I32 with the
// matching -DHDC_MR_NAME=run_map_reduce_f32|...), splitting the largest kernel
// family over four translation units.
#include "hdc_launch.hpp"

#if !defined(HDC_MR_STORAGE) || !defined(HDC_MR_NAME)
#error "define HDC_MR_STORAGE and HDC_MR_NAME"
#endif

namespace hdc {

hdc_status HDC_MR_NAME(const hdc_functor& fm, const hdc_functor& f, const void* x, void* y, int64_t n,
                       hdc_accum acc, void* out, void* ws, uint64_t* ticket, const Tuning& t, hipStream_t st) {
  using S = HDC_MR_STORAGE;
  if constexpr (std::is_same_v<S, I32>) {
    (void)acc;
    return with_int_fn(f, [&](auto fn) {
      return with_int_fn(fm, [&](auto mfn) {
        return launch_reduce<decltype(fn), I32, IntAcc, decltype(mfn), true>(fn, x, nullptr, n, out, ws, ticket, t,
                                                                             st, mfn, y);
      });
    });
  } else {
    if constexpr (std::is_same_v<S, F16>) {
      if (acc == HDC_ACC_EXACT)  // checked on entry: the fold callable is IDENTITY
        return with_float_fn(fm, [&](auto mfn) -> hdc_status {
          using FM = decltype(mfn);
          if constexpr (FM::binary)
            return fail(HDC_ERR_UNSUPPORTED, "PRODUCT cannot be mapped");
          else
            return launch_reduce<Identity, F16, ExactAcc, FM, true>(Identity{}, x, nullptr, n, out, ws, ticket, t,
                                                                   st, mfn, y);
        });
    }
    return with_float_fn(f, [&](auto fn) -> hdc_status {
      using F = decltype(fn);
      if constexpr (F::binary) {
        return fail(HDC_ERR_UNSUPPORTED, "map_reduce folds one operand");
      } else {
        return with_float_fn(fm, [&](auto mfn) -> hdc_status {
          using FM = decltype(mfn);
          if constexpr (FM::binary) {
            return fail(HDC_ERR_UNSUPPORTED, "PRODUCT cannot be mapped");
          } else {
            if (acc == HDC_ACC_COMPENSATED)
              return launch_reduce<F, S, CompAcc, FM, true>(fn, x, nullptr, n, out, ws, ticket, t, st, mfn, y);
            return launch_reduce<F, S, PlainAcc, FM, true>(fn, x, nullptr, n, out, ws, ticket, t, st, mfn, y);
          }
        });
      }
    });
  }
}

}  // namespace hdc
